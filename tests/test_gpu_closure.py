"""GPU learned-closure kernels vs the oracle: residual generation (pairs,
features, normalised residuals), the BF16 matrix-core network's forward
pass and per-step gradients (against the FP64 oracle with the same bfloat16
rounding points), the Adam update, and that training on the method's own
residuals lowers the loss."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from paper_1211_2293_amd import treecode, workloads
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _ctx(w, lc=16):
    tc = treecode.Treecode(3, leaf_cap=lc)
    pos, mass = to_dev(w.pos), to_dev(w.mass)
    tc.build(pos, mass)
    tc.moments()
    return tc, (pos, mass)


@pytest.fixture(scope="module")
def plummer():
    w = workloads.plummer_sphere(20000, seed=90)
    tc, keep = _ctx(w)
    return w, tc, keep


def test_residuals_match_oracle(plummer):
    w, tc, _ = plummer
    targets = workloads.sample_indices(w.n, 64, seed=203)
    feat, y, cell = tc.residuals(0.9, 1e-2, to_dev(targets.astype(np.int32)))
    feat, y, cell = feat.cpu().numpy(), y.cpu().numpy(), cell.cpu().numpy()
    t = oracle.Tree(w.pos, w.mass, 16)
    r = t.residuals(0.9, 1e-2, targets)
    assert len(cell) == len(r["cell"]) and len(cell) > 64 * 50
    off = np.concatenate([[0], np.cumsum(r["count"])])
    for k in range(len(targets)):
        a, b = off[k], off[k + 1]
        og = np.argsort(cell[a:b])
        oo = np.argsort(r["cell"][a:b])
        np.testing.assert_array_equal(cell[a:b][og], r["cell"][a:b][oo])
        np.testing.assert_allclose(feat[a:b][og], r["feat"][a:b][oo], rtol=1e-6, atol=1e-6)
        ref = r["y"][a:b][oo]
        assert np.all(np.abs(y[a:b][og] - ref) <= 1e-6 * np.abs(ref) + 1e-9)


def _features(n=3000, seed=91):
    rng = np.random.default_rng(seed)
    f = np.concatenate([rng.normal(size=(n, 9)) * [1, 1, 1, .3, .3, .3, .3, .3, .3],
                        rng.uniform(0, 8, (n, 1))], axis=1).astype(np.float32)
    y = (rng.normal(size=(n, 3)) * 0.02).astype(np.float32)
    return f, y


def test_forward_matches_bf16_oracle(plummer):
    _, tc, _ = plummer
    theta = mlp.init_params(seed=5)
    tc.mlp_load(to_dev(theta))
    f, _ = _features()
    out = tc.mlp_forward(to_dev(f)).cpu().numpy()
    ref, _ = mlp.forward(theta, f, bf16_ops=True)
    print(f"forward rel L2 {oracle.rel_l2(out, ref):.2e}", flush=True)
    assert oracle.rel_l2(out, ref) < 1e-3
    np.testing.assert_array_equal(tc.mlp_get().cpu().numpy(), theta)


def test_gradient_matches_bf16_oracle(plummer):
    _, tc, _ = plummer
    theta = mlp.init_params(seed=6)
    tc.mlp_load(to_dev(theta))
    f, y = _features(4000, seed=92)
    idx = np.random.default_rng(93).permutation(4000)[:2500].astype(np.int32)
    grad = torch.empty(mlp.NPARAM, dtype=torch.float32, device="cuda")
    loss = tc.mlp_step(to_dev(f), to_dev(y), to_dev(idx), lr=0.0, grad=grad)
    rl, rg = mlp.loss_and_grad(theta, f[idx], y[idx], bf16_ops=True)
    g = grad.cpu().numpy()
    print(f"loss {loss:.6e} vs {rl:.6e}; grad rel L2 {oracle.rel_l2(g, rg):.2e}", flush=True)
    assert abs(loss - rl) <= 1e-4 * rl
    assert oracle.rel_l2(g, rg) < 1e-3
    # lr = 0 leaves the parameters unchanged
    np.testing.assert_array_equal(tc.mlp_get().cpu().numpy(), theta)


def test_adam_step_matches_oracle(plummer):
    _, tc, _ = plummer
    theta = mlp.init_params(seed=7)
    tc.mlp_load(to_dev(theta))
    f, y = _features(1000, seed=94)
    grad = torch.empty(mlp.NPARAM, dtype=torch.float32, device="cuda")
    tc.mlp_step(to_dev(f), to_dev(y), lr=1e-3, grad=grad)
    g = grad.cpu().numpy().astype(np.float64)
    ref, _, _ = mlp.adam(theta.astype(np.float64), g, np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), 1, lr=1e-3)
    np.testing.assert_allclose(tc.mlp_get().cpu().numpy(), ref, rtol=0, atol=2e-6)


def test_training_on_residuals_lowers_the_loss():
    from paper_1211_2293_amd import closure
    w = workloads.plummer_sphere(65536, seed=95)
    tc, keep = _ctx(w)
    f_tr, y_tr = closure.residual_pairs(tc, 0.9, 1e-2, workloads.sample_indices(w.n, 512, seed=203))
    f_va, y_va = closure.residual_pairs(tc, 0.9, 1e-2, workloads.sample_indices(w.n, 128, seed=204))
    st = closure.train(tc, f_tr, y_tr, epochs=40, val=(f_va, y_va))
    print(f"pairs {st['pairs']}, {st['steps']} steps; loss {st['loss_first']:.3e} -> {st['loss_last']:.3e}; "
          f"validation {st['val_mse']:.3e} vs zero predictor {st['val_mse_zero']:.3e}", flush=True)
    assert st["loss_last"] < 0.5 * st["loss_first"]
    assert st["val_mse"] < 0.5 * st["val_mse_zero"]


@pytest.fixture(scope="module")
def learned_case():
    """A 4000-body Plummer sphere, a random network scaled so corrections
    stay a few percent of the force, and the oracle's learned walk."""
    w = workloads.plummer_sphere(4000, seed=97)
    tc, keep = _ctx(w)
    p = mlp.unflatten(mlp.init_params(seed=9).astype(np.float64))
    p["W3"] *= 0.2
    theta = mlp.flatten(p).astype(np.float32)
    tc.mlp_load(to_dev(theta))
    t = oracle.Tree(w.pos, w.mass, 16)
    ref = mlp.learned_corrections(t, 0.9, 0.5, theta, G=1.0)
    return w, tc, keep, t, theta, ref


def test_learned_walk_tau_zero_is_plain_walk_at_theta_p(learned_case):
    w, tc, _, t, _, ref = learned_case
    acc, pot = tc.forces_learned(0.9, 0.5, 0.0, eps=1e-2)
    m2p, p2p = (v.cpu().numpy() for v in tc.counts())
    kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
    gb, gc = t.groups(64, 1024)
    rm2p, rp2p = t.walk_counts_groups(0.5, gb, gc)
    np.testing.assert_array_equal(m2p, rm2p)
    np.testing.assert_array_equal(p2p, rp2p)
    assert np.all(kept == 0)
    np.testing.assert_array_equal(fell, ref["per_group"])
    a, ph = t.forces_groups(0.5, gb, gc, eps=1e-2)
    ea, ep = oracle.rel_l2(acc.cpu().numpy(), a), oracle.rel_l2(pot.cpu().numpy(), ph)
    print(f"tau=0: acc {ea:.2e} pot {ep:.2e}; learned cells {ref['per_group'].sum()}", flush=True)
    assert ea < 1e-5 and ep < 1e-5


def test_learned_walk_tau_inf_is_theta_l_plus_corrections(learned_case):
    w, tc, _, t, _, ref = learned_case
    acc, pot = tc.forces_learned(0.9, 0.5, float("inf"), eps=1e-2)
    m2p, p2p = (v.cpu().numpy() for v in tc.counts())
    kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
    gb, gc = t.groups(64, 1024)
    rm2p, rp2p = t.walk_counts_groups(0.9, gb, gc)
    np.testing.assert_array_equal(m2p, rm2p)
    np.testing.assert_array_equal(p2p, rp2p)
    np.testing.assert_array_equal(kept, ref["per_group"])
    assert np.all(fell == 0)
    a, ph = t.forces_groups(0.9, gb, gc, eps=1e-2)
    g_acc = acc.cpu().numpy()
    total = oracle.rel_l2(g_acc, a + ref["corr"])
    corr = oracle.rel_l2(g_acc - a, ref["corr"])
    ep = oracle.rel_l2(pot.cpu().numpy(), ph)
    size = np.linalg.norm(ref["corr"]) / np.linalg.norm(a)
    print(f"tau=inf: total {total:.2e}, corrections {corr:.2e} (|corr|/|acc| {size:.2e}), pot {ep:.2e}", flush=True)
    assert size > 1e-3
    assert corr < 1e-2 and total < 1e-5 + 1e-2 * size and ep < 1e-5


def test_learned_walk_fallback_decisions(learned_case):
    """For a tau between the extremes every learned cell is either kept or
    falls back (their sum per group does not depend on tau), and a cell
    falls back exactly when the group's largest |yhat| exceeds tau (up to
    ties within the network's rounding)."""
    w, tc, _, t, _, ref = learned_case
    gm, pg = ref["pair_gmax"], ref["pair_group"]
    tau = float(np.median(gm))
    acc, _ = tc.forces_learned(0.9, 0.5, tau, eps=1e-2)
    kept, fell = (v.cpu().numpy() for v in tc.learned_counts())
    np.testing.assert_array_equal(kept + fell, ref["per_group"])
    sure_fall = np.bincount(pg[gm > tau * 1.01], minlength=len(kept))
    sure_keep = np.bincount(pg[gm < tau * 0.99], minlength=len(kept))
    assert np.all(fell >= sure_fall) and np.all(kept >= sure_keep)
    print(f"tau={tau:.3f}: kept {kept.sum()} fell {fell.sum()}", flush=True)
    assert kept.sum() > 0 and fell.sum() > 0
    assert np.all(np.isfinite(acc.cpu().numpy()))

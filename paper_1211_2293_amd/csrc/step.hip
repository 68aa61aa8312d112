// Time step and diagnostics.  §3.1 ends the algorithm with each body
// updating its position and velocity from the computed forces; the update
// here is the kick-drift-kick leapfrog.  The diagnostics are FP64 sums with
// a fixed reduction tree, so they are bit-reproducible run to run.
#include "tc_internal.h"

namespace tc {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_kick_drift(T* __restrict__ pos, T* __restrict__ vel,
                                                    const float* __restrict__ acc, int64_t nd, T hdt, T dt) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nd;
         j += (int64_t)gridDim.x * blockDim.x) {
        const T v = vel[j] + hdt * (T)acc[j];
        vel[j] = v;
        pos[j] = pos[j] + dt * v;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_kick(T* __restrict__ vel, const float* __restrict__ acc, int64_t nd, T hdt) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nd;
         j += (int64_t)gridDim.x * blockDim.x)
        vel[j] = vel[j] + hdt * (T)acc[j];
}

// Per-block partial sums of the 8 diagnostics: grid-stride accumulation in
// a fixed order per thread, then a fixed LDS tree.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_diag_part(const T* __restrict__ mass, const T* __restrict__ vel,
                                                   const float* __restrict__ acc, const float* __restrict__ pot,
                                                   int64_t n, double* __restrict__ part) {
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double m = (double)mass[i];
        double v2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double v = (double)vel[i * D + a];
            v2 = v2 + v * v;
            s[2 + a] = s[2 + a] + m * v;
            s[5 + a] = s[5 + a] + m * (double)acc[i * D + a];
        }
        s[0] = s[0] + m * v2;
        s[1] = s[1] + m * (double)pot[i];
    }
    __shared__ double sh[8][256];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) sh[q][t] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < 8; ++q) sh[q][t] = sh[q][t] + sh[q][t + w];
        __syncthreads();
    }
    if (t < 8) part[blockIdx.x * 8 + t] = sh[t][0];
}

__global__ void __launch_bounds__(256) k_diag_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double sh[8][256];
    const int t = threadIdx.x;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = t; b < nb; b += 256)
        for (int q = 0; q < 8; ++q) s[q] = s[q] + part[b * 8 + q];
    for (int q = 0; q < 8; ++q) sh[q][t] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 8; ++q) sh[q][t] = sh[q][t] + sh[q][t + w];
        __syncthreads();
    }
    if (t < 8) out[t] = (t < 2 ? 0.5 : 1.0) * sh[t][0];
}

}  // namespace

hipError_t launch_kick_drift(void* pos, void* vel, const float* acc, int64_t n, int dim, int f64,
                             double dt, hipStream_t s) {
    const int64_t nd = n * dim;
    const unsigned nb = grid_for(nd, 8192);
    if (f64)
        hipLaunchKernelGGL(k_kick_drift<double>, dim3(nb), dim3(256), 0, s, (double*)pos, (double*)vel, acc, nd,
                           0.5 * dt, dt);
    else
        hipLaunchKernelGGL(k_kick_drift<float>, dim3(nb), dim3(256), 0, s, (float*)pos, (float*)vel, acc, nd,
                           (float)(0.5 * dt), (float)dt);
    return hipGetLastError();
}

hipError_t launch_kick(void* vel, const float* acc, int64_t n, int dim, int f64, double dt, hipStream_t s) {
    const int64_t nd = n * dim;
    const unsigned nb = grid_for(nd, 8192);
    if (f64)
        hipLaunchKernelGGL(k_kick<double>, dim3(nb), dim3(256), 0, s, (double*)vel, acc, nd, 0.5 * dt);
    else
        hipLaunchKernelGGL(k_kick<float>, dim3(nb), dim3(256), 0, s, (float*)vel, acc, nd, (float)(0.5 * dt));
    return hipGetLastError();
}

hipError_t launch_diag(const void* mass, const void* vel, const float* acc, const float* pot,
                       int64_t n, int dim, int f64, double* part, double* out, hipStream_t s) {
    const unsigned nb = kDiagBlocks;
    if (f64) {
        if (dim == 3) hipLaunchKernelGGL((k_diag_part<double, 3>), dim3(nb), dim3(256), 0, s, (const double*)mass, (const double*)vel, acc, pot, n, part);
        else hipLaunchKernelGGL((k_diag_part<double, 2>), dim3(nb), dim3(256), 0, s, (const double*)mass, (const double*)vel, acc, pot, n, part);
    } else {
        if (dim == 3) hipLaunchKernelGGL((k_diag_part<float, 3>), dim3(nb), dim3(256), 0, s, (const float*)mass, (const float*)vel, acc, pot, n, part);
        else hipLaunchKernelGGL((k_diag_part<float, 2>), dim3(nb), dim3(256), 0, s, (const float*)mass, (const float*)vel, acc, pot, n, part);
    }
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, (const double*)part, (int)nb, out);
    return hipGetLastError();
}

}  // namespace tc

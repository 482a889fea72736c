// Device helpers of the dual phase (reductions, per-row work), shared by the
// single-instance and the batched kernels.
#pragma once

#include <cfloat>

#include "common.hpp"

namespace cblp {
namespace dual {

constexpr int NR = 8;   // P, c.eta, infeasibility, Polyak norm, theta, ||eta||^2, Z, sum c
enum { R_P = 0, R_CETA, R_INF, R_G, R_TH, R_E2, R_Z, R_CS };

// relative infeasibility sum (u - c)^+ / sum c (the plain sum when sum c = 0)
__device__ __forceinline__ double rel_infeas(const double (&x)[NR])
{
    return x[R_CS] > 0.0 ? x[R_INF] / x[R_CS] : x[R_INF];
}

// Deterministic block reduction of NR values (R_TH is a minimum, the rest
// sums): a shuffle tree inside each wave, then every thread folds the wave
// results in wave order.  sh holds NR * blockDim/64 doubles.
__device__ void block_reduce(double (&x)[NR], double* sh)
{
#pragma unroll
    for (int q = 0; q < NR; ++q)
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_down(x[q], o, 64);
            x[q] = q == R_TH ? fmin(x[q], y) : x[q] + y;
        }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (int)(blockDim.x >> 6);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NR; ++q) sh[q * 16 + wave] = x[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        double r = sh[q * 16];
        for (int w = 1; w < nw; ++w) r = q == R_TH ? fmin(r, sh[q * 16 + w]) : r + sh[q * 16 + w];
        x[q] = r;
    }
}

__device__ __forceinline__ void clear(double (&x)[NR])
{
#pragma unroll
    for (int q = 0; q < NR; ++q) x[q] = 0.0;
    x[R_TH] = 1.0;
}

template <typename T, typename Args>
__device__ __forceinline__ void row_work(const Args& a, int64_t i, double u, long long cnt1,
                                         double (&x)[NR])
{
    const T* c = (const T*)a.c;
    const T* eta = (const T*)a.eta;
    const T* tauv = (const T*)a.tau_vec;
    a.u_d[i] = u;
    const double ci = (double)c[i], ei = (double)eta[i];
    const double g = u - ci;
    x[R_CETA] += ci * ei;
    x[R_CS] += ci;
    x[R_E2] += ei * ei;
    if (g > 0.0) x[R_INF] += g;
    const double ti = tauv ? (double)tauv[i] : a.tau_s;
    const double gh = (ei <= 0.0 && g < 0.0) ? 0.0 : g;
    x[R_G] += ti * gh * gh;
    if (a.mode == 0) {
        const double su = a.sum_u[i] + u;
        a.sum_u[i] = su;
        const double ub = su / (double)cnt1;
        if (ub > ci) x[R_TH] = fmin(x[R_TH], ci / ub);
    }
}

__device__ __forceinline__ void store_part(double* p, const double (&x)[NR])
{
#pragma unroll
    for (int q = 0; q < NR; ++q) p[q] = x[q];
}

}  // namespace dual
}  // namespace cblp

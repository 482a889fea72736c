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

__device__ __forceinline__ void clear(double (&x)[NR])
{
#pragma unroll
    for (int q = 0; q < NR; ++q) x[q] = 0.0;
    x[R_TH] = 1.0;
}

// The shuffle tree of one wave: lane 0 ends with the wave's NR values
// (R_TH a minimum, the rest sums).
__device__ __forceinline__ void wave_reduce(double (&x)[NR])
{
#pragma unroll
    for (int q = 0; q < NR; ++q)
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_down(x[q], o, 64);
            x[q] = q == R_TH ? fmin(x[q], y) : x[q] + y;
        }
}

// Deterministic block reduction of NR values: the shuffle tree inside each
// wave, then every thread folds the results of waves [0, nw) in wave order
// (nw <= 16; every wave of the block takes part).  sh holds NR * 16 doubles.
__device__ void block_reduce(double (&x)[NR], double* sh, int nw)
{
    wave_reduce(x);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
__device__ __forceinline__ void block_reduce(double (&x)[NR], double* sh)
{
    block_reduce(x, sh, (int)(blockDim.x >> 6));
}

// x combined with y: R_TH by minimum, the rest by sums
__device__ __forceinline__ void combine(double (&x)[NR], const double (&y)[NR])
{
#pragma unroll
    for (int r = 0; r < NR; ++r) x[r] = r == R_TH ? fmin(x[r], y[r]) : x[r] + y[r];
}

// The fold of partials of 64 consecutive products (library order), q in
// [0, nf): four at a time in order, which is a 256-product block's
// block_reduce (its four waves' sums folded in wave order), then those
// strided over the first 256 threads; every thread of the block calls this,
// and all get the sums (R_Z left 0).  sh as block_reduce.
__device__ void fold_partials(const double* part, int nf, double (&x)[NR], double* sh)
{
    clear(x);
    if (threadIdx.x < 256)
        for (int g = (int)threadIdx.x; g < (nf + 3) / 4; g += 256) {
            double y[NR];
            for (int k = 0; k < 4; ++k) {
                const int q = 4 * g + k;
                double p[NR];
                clear(p);   // past the last product: the values of empty waves
                if (q < nf)
                    for (int r = 0; r < NR; ++r)
                        if (r != R_Z) p[r] = part[(size_t)q * 8 + r];
                if (k == 0)
                    for (int r = 0; r < NR; ++r) y[r] = p[r];
                else
                    combine(y, p);
            }
            combine(x, y);
        }
    block_reduce(x, sh, 4);
}

// The per-row work on loaded values: ci = c_i, ei = eta_i, ti = tau_i,
// su = sum_u_i before this iteration; returns the new sum_u_i (mode 0).
__device__ __forceinline__ double row_work_values(double ci, double ei, double ti, double su,
                                                  double u, long long cnt1, int mode,
                                                  double (&x)[NR])
{
    const double g = u - ci;
    x[R_CETA] += ci * ei;
    x[R_CS] += ci;
    x[R_E2] += ei * ei;
    if (g > 0.0) x[R_INF] += g;
    const double gh = (ei <= 0.0 && g < 0.0) ? 0.0 : g;
    x[R_G] += ti * gh * gh;
    if (mode == 0) {
        su = su + u;
        const double ub = su / (double)cnt1;
        if (ub > ci) x[R_TH] = fmin(x[R_TH], ci / ub);
    }
    return su;
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
    const double ti = tauv ? (double)tauv[i] : a.tau_s;
    const double su = row_work_values(ci, ei, ti, a.mode == 0 ? a.sum_u[i] : 0.0, u, cnt1, a.mode, x);
    if (a.mode == 0) a.sum_u[i] = su;
}

__device__ __forceinline__ void store_part(double* p, const double (&x)[NR])
{
#pragma unroll
    for (int q = 0; q < NR; ++q) p[q] = x[q];
}

}  // namespace dual
}  // namespace cblp

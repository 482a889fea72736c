// Stochastic minibatch SPFOM (Algorithm 2, Section 4.1; Algorithm 3 with
// k B < L, Section 4.3): each iteration re-solves only the B segments the
// caller sampled, keeps every other segment's sales from the last time it
// was solved, and steps the duals with the sales of all segments.
//
// State kept by the handle (made on first use, cleared by spfom_reset):
//   yq [nnz]     each entry's current sale in fixed-point quanta (row-major
//                library copy order); 0 initially (y^0 = 0)
//   S_run [n]    sum over segments of yq, as 64-bit integers, kept by adding
//                each re-solved entry's change (exact, order-free)
//   stamp [L]    the last iteration that sampled each segment (rejects a
//                segment listed twice in one iteration)
//
// k_minibatch: an 8-lane group per sampled segment over the row-major copy.
// Its inner solve takes the same steps, in the same rounding, as the
// full-batch kernels' (Dinkelbach from the segment's last R*, sums in the
// 8-lane order, the same cycle rule), so B = L gives the full batch's bits.
#include "segment_core.hpp"

namespace cblp {
namespace {

using seg::fmadd;
using seg::group_sum;
using seg::quantum;
using seg::ratio;

template <typename T>
__global__ void __launch_bounds__(256) k_minibatch(MbArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H] signed changes of the head products
    const int H = a.H;
    for (int j = threadIdx.x; j < H; j += 256) bins[j] = 0ull;
    __syncthreads();
    const int g = threadIdx.x & (kGroup - 1);
    const int lane = threadIdx.x & 63;
    const T* __restrict__ rho = (const T*)a.rho;
    const T* __restrict__ v2 = (const T*)a.v2;
    const T* __restrict__ d2 = (const T*)a.den2;
    const int groups = 256 / kGroup;
    for (int64_t q = (int64_t)blockIdx.x * groups + threadIdx.x / kGroup; q < a.B;
         q += (int64_t)gridDim.x * groups) {
        const int32_t l = a.batch[q];
        if (l < 0 || (int64_t)l >= a.L) {            // rejected; the host reports it
            if (g == 0) atomicOr(a.err, 1u);
            continue;
        }
        if (g == 0 && atomicExch(&a.stamp[l], a.it) == a.it) atomicOr(a.err, 2u);
        const int64_t p = a.inv_perm[l];
        const int64_t b = a.ptr2[p];
        const int k = (int)(a.ptr2[p + 1] - b);
        const T vt0 = ((const T*)a.vt0)[p];
        const T lam = ((const T*)a.lam)[p];
        // Dinkelbach, as the full-batch kernels take it (their comments)
        auto full = [&](T R, T& N, T& Dn) {
            T n_ = T(0), d_ = T(0);
            for (int t = g; t < k; t += kGroup) {
                const T nn = rho[a.idx2[b + t]] * v2[b + t];
                const T dd = d2[b + t];
                const T w = nn > R * dd ? T(1) : T(0);
                n_ = fmadd(w, nn, n_);
                d_ = fmadd(w, dd, d_);
            }
            N = group_sum(n_);
            Dn = group_sum(d_);
        };
        auto changed = [&](T R, T Rn) {
            bool c = false;
            for (int t = g; t < k; t += kGroup) {
                const T nn = rho[a.idx2[b + t]] * v2[b + t];
                const T dd = d2[b + t];
                c = c || ((nn > Rn * dd) != (nn > R * dd));
            }
            return ((__ballot(c) >> (lane & 56)) & 0xFFull) != 0ull;
        };
        T R = ((const T*)a.Rwarm)[p], N, Dn;
        full(R, N, Dn);
        T Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        T pR = R, pN = N, pD = Dn, pRs = Rs;
        bool diff = false;
        const int cap = kGroup * ((k + kGroup - 1) / kGroup) + 1;
        for (int round = 0; round <= cap; ++round) {
            diff = changed(R, Rs);
            if (!diff) break;
            pR = R;
            pN = N;
            pD = Dn;
            pRs = Rs;
            R = Rs;
            full(R, N, Dn);
            Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        }
        if (diff && changed(R, Rs) && pRs > Rs) {   // still alternating: the set of larger ratio
            R = pR;
            N = pN;
            Dn = pD;
            Rs = pRs;
        }
        const T lamD = ratio(lam, vt0 + Dn) * (T)a.fx_scale;
        for (int t = g; t < k; t += kGroup) {
            const int32_t j = a.idx2[b + t];
            const T x = v2[b + t];
            const unsigned long long qn = rho[j] * x > R * d2[b + t] ? quantum(lamD, x) : 0ull;
            const unsigned long long qo = a.wide ? ((const unsigned long long*)a.yq)[b + t]
                                                 : (unsigned long long)((const unsigned*)a.yq)[b + t];
            if (qn != qo) {
                if (a.wide)
                    ((unsigned long long*)a.yq)[b + t] = qn;
                else
                    ((unsigned*)a.yq)[b + t] = (unsigned)qn;
                const unsigned long long d = qn - qo;   // two's complement change
                if (j < H)
                    atomicAdd(&bins[j], d);
                else
                    atomicAdd(&a.S_run[j], d);
            }
        }
        if (g == 0) ((T*)a.Rwarm)[p] = Rs;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < H; j += 256)
        if (bins[j]) atomicAdd(&a.S_run[j], bins[j]);
}

__global__ void k_mb_stamp_init(int64_t L, int* stamp)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L;
         l += (int64_t)gridDim.x * blockDim.x)
        stamp[l] = -1;
}

__global__ void k_mb_inv_perm(int64_t L, const int32_t* perm, int32_t* inv)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x)
        inv[perm[p]] = (int32_t)p;
}

}  // namespace

template <typename T>
hipError_t launch_minibatch(const MbArgs& a, int grid, hipStream_t s)
{
    const size_t lds = (size_t)a.H * 8;
    (void)hipFuncSetAttribute((const void*)k_minibatch<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_minibatch<T>, dim3(grid), dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_minibatch_init(int64_t L, const int32_t* perm, int32_t* inv_perm, int* stamp,
                                 hipStream_t s)
{
    if (L > 0) {
        hipLaunchKernelGGL(k_mb_stamp_init, dim3(1024), dim3(256), 0, s, L, stamp);
        hipLaunchKernelGGL(k_mb_inv_perm, dim3(1024), dim3(256), 0, s, L, perm, inv_perm);
    }
    return hipGetLastError();
}

template hipError_t launch_minibatch<float>(const MbArgs&, int, hipStream_t);
template hipError_t launch_minibatch<double>(const MbArgs&, int, hipStream_t);

}  // namespace cblp

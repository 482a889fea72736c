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
#include "minibatch.hpp"
#include "segment_core.hpp"

namespace cblp {
namespace {

using seg::fmadd;
using seg::group_sum;
using seg::quantum;
using seg::ratio;

constexpr int kRowRegs = 8;   // entries per lane held in registers (rows up to 64)

// A segment's row and own values, by caller id, in one 32-byte record (one
// line per sampled segment instead of one for each of five arrays).
template <typename T>
struct alignas(32) MbSeg {
    int64_t b;    // row start in the row-major copy
    int32_t k;    // entries
    int32_t p;    // position (the warm start's slot)
    T vt0, lam;
};
static_assert(sizeof(MbSeg<float>) == kMbRecBytes && sizeof(MbSeg<double>) == kMbRecBytes,
              "record size");

// An entry's product id, v, denominator weight and kept sale in one record,
// so a sampled row is one run of lines rather than one in each of four arrays.
template <typename T>
struct MbEnt;
template <>
struct alignas(16) MbEnt<float> {
    int32_t j;
    float v, d;
    unsigned q;
};
template <>
struct alignas(32) MbEnt<double> {
    int32_t j, pad;
    double v, d;
    unsigned long long q;
};
static_assert(sizeof(MbEnt<float>) == mb_ent_bytes<float>() &&
                  sizeof(MbEnt<double>) == mb_ent_bytes<double>(),
              "entry record size");

// threads per block: FP32 runs one 1024-thread block per CU (4 waves per
// SIMD at its register count) with up to 16,384 bins; FP64, whose solve needs
// more registers, 256-thread blocks with up to 8,192
template <typename T>
constexpr int mb_threads() { return sizeof(T) == 4 ? 1024 : 256; }

template <typename T>
__global__ void __launch_bounds__(mb_threads<T>()) k_minibatch(MbArgs a)
{
    constexpr int NT = mb_threads<T>();
    extern __shared__ unsigned long long bins[];   // [a.H] signed changes of the head products
    const int H = a.H;
    for (int j = threadIdx.x; j < H; j += NT) bins[j] = 0ull;
    __syncthreads();
    const int g = threadIdx.x & (kGroup - 1);
    const int lane = threadIdx.x & 63;
    const T* __restrict__ rho = (const T*)a.rho;
    MbEnt<T>* __restrict__ ent = (MbEnt<T>*)a.ent;
    const int groups = NT / kGroup;
    // Each group walks its segments q, q + qs, ...  The chain that locates a
    // segment's row (its id, then its record) runs ahead of the solve: while
    // segment q is solved, the id of q + 2 qs and the record of q + qs load.
    using Q = decltype(MbEnt<T>::q);
    const int64_t qs = (int64_t)gridDim.x * groups;
    const int64_t q0 = (int64_t)blockIdx.x * groups + threadIdx.x / kGroup;
    auto ok = [&](int32_t l) { return l >= 0 && (int64_t)l < a.L; };
    auto id = [&](int64_t q) { return q < a.B ? a.batch[q] : (int32_t)-1; };
    const MbSeg<T>* __restrict__ rec = (const MbSeg<T>*)a.rec;
    int32_t lc = id(q0), ln = id(q0 + qs);
    MbSeg<T> rc{};
    if (ok(lc)) rc = rec[lc];
    for (int64_t q = q0; q < a.B; q += qs) {
        const int32_t l = lc;
        const MbSeg<T> r = rc;
        {   // advance the chain
            const int32_t l2 = id(q + 2 * qs);
            if (ok(ln)) rc = rec[ln];
            lc = ln;
            ln = l2;
        }
        if (!ok(l)) {                                // rejected; the host reports it
            if (g == 0) atomicOr(a.err, 1u);
            continue;
        }
        if (g == 0 && atomicExch(&a.stamp[l], a.it) == a.it) atomicOr(a.err, 2u);
        const int64_t p = r.p, b = r.b;
        const int k = r.k;
        const T vt0 = r.vt0, lam = r.lam;
        // a row of at most kRowRegs * kGroup entries is held in registers (ids,
        // v, rho_j v, the denominator weight and the kept sale), so the rounds
        // below read it once
        const bool held = k <= kRowRegs * kGroup;
        int32_t hj[kRowRegs];
        T hv[kRowRegs], hn[kRowRegs], hd[kRowRegs];
        Q hq[kRowRegs];
        if (held) {
#pragma unroll
            for (int u = 0; u < kRowRegs; ++u) {
                const int t = g + u * kGroup;
                const MbEnt<T> e = t < k ? ent[b + t] : MbEnt<T>{};
                hj[u] = e.j;
                hv[u] = e.v;
                hd[u] = e.d;
                hq[u] = e.q;
            }
#pragma unroll
            for (int u = 0; u < kRowRegs; ++u)
                hn[u] = g + u * kGroup < k ? rho[hj[u]] * hv[u] : T(0);
        }
        // Dinkelbach, as the full-batch kernels take it (their comments); the
        // held and the streamed forms add the same terms in the same order
        auto full = [&](T R, T& N, T& Dn) {
            T n_ = T(0), d_ = T(0);
            if (held) {
#pragma unroll
                for (int u = 0; u < kRowRegs; ++u)
                    if (g + u * kGroup < k) {
                        const T w = hn[u] > R * hd[u] ? T(1) : T(0);
                        n_ = fmadd(w, hn[u], n_);
                        d_ = fmadd(w, hd[u], d_);
                    }
            } else {
                for (int t = g; t < k; t += kGroup) {
                    const T nn = rho[ent[b + t].j] * ent[b + t].v;
                    const T dd = ent[b + t].d;
                    const T w = nn > R * dd ? T(1) : T(0);
                    n_ = fmadd(w, nn, n_);
                    d_ = fmadd(w, dd, d_);
                }
            }
            N = group_sum(n_);
            Dn = group_sum(d_);
        };
        auto changed = [&](T R, T Rn) {
            bool c = false;
            if (held) {
#pragma unroll
                for (int u = 0; u < kRowRegs; ++u)
                    if (g + u * kGroup < k)
                        c = c || ((hn[u] > Rn * hd[u]) != (hn[u] > R * hd[u]));
            } else {
                for (int t = g; t < k; t += kGroup) {
                    const T nn = rho[ent[b + t].j] * ent[b + t].v;
                    const T dd = ent[b + t].d;
                    c = c || ((nn > Rn * dd) != (nn > R * dd));
                }
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
        // each entry's new quantum against its kept one; the change goes to
        // the block's bins (head products) or the global totals
        auto sale = [&](int t, int32_t j, T v, bool in, Q qo) {
            const unsigned long long qn = in ? quantum(lamD, v) : 0ull;
            if (qn != (unsigned long long)qo) {
                ent[b + t].q = (Q)qn;
                const unsigned long long d = qn - (unsigned long long)qo;
                if (j < H)
                    atomicAdd(&bins[j], d);   // two's complement change
                else
                    atomicAdd(&a.S_run[j], d);
            }
        };
        if (held) {
#pragma unroll
            for (int u = 0; u < kRowRegs; ++u) {
                const int t = g + u * kGroup;
                if (t < k) sale(t, hj[u], hv[u], hn[u] > R * hd[u], hq[u]);
            }
        } else {
            for (int t = g; t < k; t += kGroup) {
                const MbEnt<T> e = ent[b + t];
                sale(t, e.j, e.v, rho[e.j] * e.v > R * e.d, e.q);
            }
        }
        if (g == 0) ((T*)a.Rwarm)[p] = Rs;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < H; j += NT)
        if (bins[j]) atomicAdd(&a.S_run[j], bins[j]);
}

template <typename T>
__global__ void k_mb_entries(int64_t nnz, const int32_t* idx2, const T* v2, const T* den2,
                             MbEnt<T>* ent)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        MbEnt<T> r{};
        r.j = idx2[e];
        r.v = v2[e];
        r.d = den2[e];
        r.q = 0;   // y^0 = 0
        ent[e] = r;
    }
}

__global__ void k_mb_stamp_init(int64_t L, int* stamp)
{
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L;
         l += (int64_t)gridDim.x * blockDim.x)
        stamp[l] = -1;
}

template <typename T>
__global__ void k_mb_records(int64_t L, const int32_t* perm, const int64_t* ptr2, const T* vt0,
                             const T* lam, MbSeg<T>* rec)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x) {
        MbSeg<T> r;
        r.b = ptr2[p];
        r.k = (int32_t)(ptr2[p + 1] - r.b);
        r.p = (int32_t)p;
        r.vt0 = vt0[p];
        r.lam = lam[p];
        rec[perm[p]] = r;
    }
}

}  // namespace

template <typename T>
int minibatch_bins(int64_t n)
{
    return (int)std::min<int64_t>(n, sizeof(T) == 4 ? 16384 : 8192);
}

template <typename T>
hipError_t launch_minibatch(const MbArgs& a, hipStream_t s)
{
    constexpr int NT = mb_threads<T>();
    const int groups = NT / kGroup;
    const int64_t cap = NT == 1024 ? 256 : 1024;   // about one wave of blocks
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.B + groups - 1) / groups, cap));
    const size_t lds = (size_t)a.H * 8;
    hipError_t e = hipFuncSetAttribute((const void*)k_minibatch<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_minibatch<T>, dim3(grid), dim3(NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_minibatch_init(int64_t L, int* stamp, hipStream_t s)
{
    if (L > 0) hipLaunchKernelGGL(k_mb_stamp_init, dim3(1024), dim3(256), 0, s, L, stamp);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_minibatch_records(int64_t L, const int32_t* perm, const int64_t* ptr2,
                                    const void* vt0, const void* lam, void* rec, int64_t nnz,
                                    const int32_t* idx2, const void* v2, const void* den2,
                                    void* ent, hipStream_t s)
{
    if (L > 0)
        hipLaunchKernelGGL(k_mb_records<T>, dim3(1024), dim3(256), 0, s, L, perm, ptr2,
                           (const T*)vt0, (const T*)lam, (MbSeg<T>*)rec);
    if (nnz > 0)
        hipLaunchKernelGGL(k_mb_entries<T>, dim3(2048), dim3(256), 0, s, nnz, idx2,
                           (const T*)v2, (const T*)den2, (MbEnt<T>*)ent);
    return hipGetLastError();
}

template int minibatch_bins<float>(int64_t);
template int minibatch_bins<double>(int64_t);
template hipError_t launch_minibatch<float>(const MbArgs&, hipStream_t);
template hipError_t launch_minibatch<double>(const MbArgs&, hipStream_t);
template hipError_t launch_minibatch_records<float>(int64_t, const int32_t*, const int64_t*,
                                                   const void*, const void*, void*, int64_t,
                                                   const int32_t*, const void*, const void*,
                                                   void*, hipStream_t);
template hipError_t launch_minibatch_records<double>(int64_t, const int32_t*, const int64_t*,
                                                    const void*, const void*, void*, int64_t,
                                                    const int32_t*, const void*, const void*,
                                                    void*, hipStream_t);

}  // namespace cblp

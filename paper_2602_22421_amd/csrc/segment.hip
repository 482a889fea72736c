// Single-instance segment kernels: the per-segment primal step over every
// segment of the library's slot-major copy and the sales scatter (device
// code in segment_core.hpp).  Two kernels ship:
//   k_segments_mixed3  FP32: rows of at most 16 entries solved by 2-lane
//                      groups, of at most 32 by 4-lane groups, longer ones
//                      by 8-lane groups; the prices in LDS, or only the
//                      popular head of them when all do not fit (SPLIT)
//   k_segments_slots   FP64: 8-lane groups, 4 register slots per lane, the
//                      prices gathered from global memory
#include "segment_core.hpp"

#include <type_traits>

namespace cblp {
namespace {

// Clear the block's LDS bins (64-bit and 32-bit ones, as 64-bit words).
__device__ __forceinline__ void clear_bins(const SegArgs& a, unsigned long long* bins)
{
    const int words = (int)(seg_bin_bytes(a.H, a.H64) / 8);
    for (int j = threadIdx.x; j < words; j += kSegThreads) bins[j] = 0ull;
}

// The block's bins leave LDS as the block's row of a.brow (plain stores;
// k_fold_rows adds the rows into the global sums, integer adds, so the order
// of the blocks does not matter).
__device__ __forceinline__ void flush_bins(const SegArgs& a, const unsigned long long* bins)
{
    const int words = (int)(seg_bin_bytes(a.H, a.H64) / 8);
    unsigned long long* row = a.brow + (int64_t)blockIdx.x * a.row_words;
    for (int w = threadIdx.x; w < words; w += kSegThreads) row[w] = bins[w];
}

// Slot-major kernel: the per-segment step over the slot-major copy (one
// contiguous 256-byte read per slot and array for a whole wave).
template <typename T, int J, bool ALL, bool LDSP, typename IdxT = int32_t, bool PSEG = false>
__global__ void __launch_bounds__(kSegThreads) k_segments_slots(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // the bins, then [a.n] prices if LDSP
    __shared__ long long zsh[kSegThreads / 64];
    T* lprice = (T*)((char*)bins + seg_bin_bytes(a.H, a.H64));
    clear_bins(a, bins);
    if (LDSP)
        for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    ZAcc zacc;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    const seg::FlatPrices<T> pr{LDSP ? (const T*)lprice : (const T*)a.rho};
    seg::process_tiles_slots<T, J, ALL, seg::FlatPrices<T>, IdxT, PSEG>(a, blockIdx.x, tiles,
                                                                        gridDim.x, bins, pr, zacc);

    __syncthreads();
    flush_bins(a, bins);
    const long long z = block_z(zacc, zsh);
    if (threadIdx.x == 0) a.zpart[blockIdx.x] = z;
}

// Three-part mixed kernel: positions [0, P2) (rows of at most 16 entries) in
// the pair layout, solved by 2-lane groups (args a2), [P2, P4) (rows of at
// most 32) in the quad layout by 4-lane groups (a4), the rest in the 8-lane
// layout (a8); each view starts at its first position.
// SPLIT: prices [0, a2.hp) in LDS, the rest from global memory.
// PSEG: also add each segment's revenue to psum (the per-segment bound).
template <typename T, typename IdxT, bool SPLIT = false, bool PSEG = false>
__global__ void __launch_bounds__(kSegThreads) k_segments_mixed3(SegArgs a2, SegArgs a4, SegArgs a8)
{
    extern __shared__ unsigned long long bins[];   // the bins, then the LDS prices
    __shared__ long long zsh[kSegThreads / 64];
    T* lprice = (T*)((char*)bins + seg_bin_bytes(a2.H, a2.H64));
    clear_bins(a2, bins);
    const int64_t np = SPLIT ? (int64_t)a2.hp : a2.n;
    for (int64_t j = threadIdx.x; j < np; j += kSegThreads) lprice[j] = ((const T*)a2.rho)[j];
    __syncthreads();

    ZAcc zacc;
    using PR = typename std::conditional<SPLIT, seg::SplitPrices<T>, seg::FlatPrices<T>>::type;
    PR pr;
    if constexpr (SPLIT)
        pr = PR{(const T*)lprice, (const T*)a2.rho, a2.hp};
    else
        pr = PR{(const T*)lprice};
    const int64_t t2 = (a2.L + seg::kPairTileRows - 1) / seg::kPairTileRows;
    seg::process_tiles_pair<T, 8, PR, IdxT, PSEG>(a2, blockIdx.x, t2, gridDim.x, bins, pr, zacc);
    const int64_t t4 = (a4.L + seg::kQuadTileRows - 1) / seg::kQuadTileRows;
    seg::process_tiles_quad<T, 8, PR, IdxT, PSEG>(a4, blockIdx.x, t4, gridDim.x, bins, pr, zacc);
    const int64_t t8 = (a8.L + kSegsPerTile - 1) / kSegsPerTile;
    seg::process_tiles_slots<T, 7, false, PR, IdxT, PSEG>(a8, blockIdx.x, t8, gridDim.x, bins, pr,
                                                          zacc);

    __syncthreads();
    flush_bins(a2, bins);
    const long long z = block_z(zacc, zsh);
    if (threadIdx.x == 0) a2.zpart[blockIdx.x] = z;
}

// Per-entry sales in the caller's CSR order from a pass that stored each
// position's threshold R and (lambda / D) 2^bits: an entry is in S* exactly
// when the segment kernel found it so (the same products and compares, in
// the same precision), and its sale is the quantum the kernel summed.
template <typename T>
__global__ void k_entry_sales(int64_t L, const int32_t* perm, const int64_t* seg_ptr,
                              const int32_t* idx, const T* v, const T* w, const int32_t* pnew,
                              const T* rho, const T* thr, const T* lamD, double inv_fx,
                              double* s_out)
{
#pragma clang fp contract(off)
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = perm[p];
        const T R = thr[p], ls = lamD[p];
        for (int64_t q = seg_ptr[l]; q < seg_ptr[l + 1]; ++q) {
            const int32_t id = idx[q];
            const T x = v[q];
            const T den = x - w[q];
            const T num = rho[pnew ? pnew[id] : id] * x;
            s_out[q] = num > R * den ? (double)(long long)seg::quantum(ls, x) * inv_fx : 0.0;
        }
    }
}

// A bound, in quanta, on the sales of each product within each segment
// block: an entry's sale lambda v / D, with D = vt0 + the sum of v - w over
// the assortment (all terms positive, the entry's own among them when it
// sells), is at most lambda v / (vt0 + v - w); scaled by 2^bits, with a
// margin far above the FP32 rounding of the kernels' quanta.  Positions map
// to blocks as in k_segments_mixed3 (the parts' tiles, dealt round robin
// over G blocks).  Ub[j * G + b] for products j < Hc.
__global__ void k_bin_bound(int64_t L, int64_t P2, int64_t P4, int G, const int64_t* ptr2,
                            const int32_t* idx2, const float* v2, const float* den2,
                            const float* vt0, const float* lam, double fx_scale, int Hc,
                            unsigned long long* Ub)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tile = p < P2 ? p / seg::kPairTileRows
                             : p < P4 ? (p - P2) / seg::kQuadTileRows
                                      : (p - P4) / kSegsPerTile;
        const int64_t b = tile % G;
        const double lp = (double)lam[p], vt = (double)vt0[p];
        for (int64_t e = ptr2[p]; e < ptr2[p + 1]; ++e) {
            const int32_t j = idx2[e];
            if (j >= Hc) continue;
            const double ub = lp * (double)v2[e] / (vt + (double)den2[e]) * fx_scale;
            atomicAdd(&Ub[(int64_t)j * G + b], (unsigned long long)(ub * (1.0 + 1.0 / 1024)) + 2ull);
        }
    }
}

// need = 1 + the largest product id whose bound reaches 2^32 in some block
// (0 if none): one product per thread.
__global__ void k_bin_need(const unsigned long long* Ub, int G, int Hc, int* need)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Hc) return;
    unsigned long long mx = 0ull;
    for (int b = 0; b < G; ++b) mx = max(mx, Ub[(int64_t)j * G + b]);
    if (mx >= (1ull << 32)) atomicMax(need, j + 1);
}

}  // namespace

hipError_t launch_bin_bound(int64_t L, int64_t P2, int64_t P4, int G, const int64_t* ptr2,
                            const int32_t* idx2, const void* v2, const void* den2,
                            const void* vt0, const void* lam, double fx_scale, int Hc,
                            unsigned long long* Ub, int* need, hipStream_t s)
{
    if (L > 0)
        hipLaunchKernelGGL(k_bin_bound, dim3(2048), dim3(256), 0, s, L, P2, P4, G, ptr2, idx2,
                           (const float*)v2, (const float*)den2, (const float*)vt0,
                           (const float*)lam, fx_scale, Hc, Ub);
    if (Hc > 0)
        hipLaunchKernelGGL(k_bin_need, dim3((unsigned)((Hc + 255) / 256)), dim3(256), 0, s, Ub, G,
                           Hc, need);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_entry_sales(int64_t L, const int32_t* perm, const int64_t* seg_ptr,
                              const int32_t* idx, const void* v, const void* w,
                              const int32_t* pnew, const void* rho, const void* thr,
                              const void* lamD, double inv_fx, double* s_out, hipStream_t s)
{
    if (L > 0)
        hipLaunchKernelGGL(k_entry_sales<T>, dim3(2048), dim3(256), 0, s, L, perm, seg_ptr, idx,
                           (const T*)v, (const T*)w, pnew, (const T*)rho, (const T*)thr,
                           (const T*)lamD, inv_fx, s_out);
    return hipGetLastError();
}

template <typename T>
const void* segment_kernel(int variant, bool pseg)
{
    // the narrow groups are FP32 kernels (eight slots of doubles would spill)
    if constexpr (sizeof(T) == 4) {
        switch (variant) {
        case kSegMixed3:
            return pseg ? (const void*)k_segments_mixed3<T, uint16_t, false, true>
                        : (const void*)k_segments_mixed3<T, uint16_t>;
        case kSegMixed3Split16:
            return pseg ? (const void*)k_segments_mixed3<T, uint16_t, true, true>
                        : (const void*)k_segments_mixed3<T, uint16_t, true>;
        case kSegMixed3Split32:
            return pseg ? (const void*)k_segments_mixed3<T, int32_t, true, true>
                        : (const void*)k_segments_mixed3<T, int32_t, true>;
        default: break;
        }
    }
    if (variant == kSegSlots16)
        return pseg ? (const void*)k_segments_slots<T, 4, true, false, uint16_t, true>
                    : (const void*)k_segments_slots<T, 4, true, false, uint16_t>;
    return pseg ? (const void*)k_segments_slots<T, 4, true, false, int32_t, true>
                : (const void*)k_segments_slots<T, 4, true, false, int32_t>;
}

template <typename T>
hipError_t launch_segments(const SegArgs& a2, const SegArgs& a4, const SegArgs& a8, int grid,
                           int variant, bool pseg, hipStream_t s)
{
    const size_t lds = seg_lds_bytes(a2.H, a2.H64, a2.n, a2.hp, sizeof(T), variant);
    const void* f = segment_kernel<T>(variant, pseg);
    // the bins' layout is per handle: allow this launch's LDS whatever another
    // handle set last
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (seg_mixed3(variant)) {
        void* args[] = {(void*)&a2, (void*)&a4, (void*)&a8};
        return hipLaunchKernel(f, dim3(grid), dim3(kSegThreads), args, lds, s);
    }
    void* args[] = {(void*)&a8};
    return hipLaunchKernel(f, dim3(grid), dim3(kSegThreads), args, lds, s);
}

template <typename T>
int segment_blocks_per_cu(int H, int H64, int64_t n, int hp, int variant)
{
    int blocks = 0;
    const size_t lds = seg_lds_bytes(H, H64, n, hp, sizeof(T), variant);
    const void* f = segment_kernel<T>(variant, false);
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, kSegThreads, lds) != hipSuccess)
        return 1;
    return blocks < 1 ? 1 : blocks;
}

template hipError_t launch_segments<float>(const SegArgs&, const SegArgs&, const SegArgs&, int, int,
                                           bool, hipStream_t);
template hipError_t launch_segments<double>(const SegArgs&, const SegArgs&, const SegArgs&, int,
                                            int, bool, hipStream_t);
template hipError_t launch_entry_sales<float>(int64_t, const int32_t*, const int64_t*,
                                              const int32_t*, const void*, const void*,
                                              const int32_t*, const void*, const void*,
                                              const void*, double, double*, hipStream_t);
template hipError_t launch_entry_sales<double>(int64_t, const int32_t*, const int64_t*,
                                               const int32_t*, const void*, const void*,
                                               const int32_t*, const void*, const void*,
                                               const void*, double, double*, hipStream_t);
template int segment_blocks_per_cu<float>(int, int, int64_t, int, int);
template int segment_blocks_per_cu<double>(int, int, int64_t, int, int);

}  // namespace cblp

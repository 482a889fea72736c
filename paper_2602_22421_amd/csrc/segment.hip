// Single-instance segment kernel: the per-segment primal step over every
// segment and the per-block LDS-bin rows of product sales (device code in
// segment_core.hpp).
#include "segment_core.hpp"

#include <type_traits>

namespace cblp {
namespace {

// The block's bins go out as one partial row (folded in block order by the
// dual phase) or, when a.part_S is null, straight into the global 64-bit
// accumulators by atomics (integer sums: the order does not matter).
__device__ __forceinline__ void flush_bins(const SegArgs& a, const unsigned long long* bins)
{
    if (a.part_S) {
        unsigned long long* out = a.part_S + (size_t)blockIdx.x * (size_t)a.H;
        for (int j = threadIdx.x; j < a.H; j += kSegThreads) out[j] = bins[j];
    } else {
        for (int j = threadIdx.x; j < a.H; j += kSegThreads)
            if (bins[j]) atomicAdd(&a.S_fx[j], bins[j]);
    }
}

// LDSP: copy the n prices into LDS behind the bins and gather from there
// (random 4-byte reads that would otherwise each take a cache-line lookup in
// the vector memory path, which the CSR stream already keeps busy).
template <typename T, int J, int DEPTH, bool LDSP>
__global__ void __launch_bounds__(kSegThreads) k_segments(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.n] prices if LDSP
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    if (LDSP)
        for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    // the grid never exceeds the tile count, except for L = 0 (one block)
    const seg::FlatPrices<T> pr{LDSP ? (const T*)lprice : (const T*)a.rho};
    seg::process_tiles<T, J, DEPTH>(a, blockIdx.x, tiles, gridDim.x, bins, pr, zacc);

    __syncthreads();
    flush_bins(a, bins);

    // block partial of sum lambda R*: fixed shuffle tree, waves in order
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Split-price kernel: the prices of the popular head [0, a.hp) are copied
// into LDS behind the bins, the rest are gathered from global memory; the
// smaller copy leaves room for more bins, so fewer sales take global atomics.
template <typename T, int J>
__global__ void __launch_bounds__(kSegThreads) k_segments_split(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.hp] prices
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    for (int j = threadIdx.x; j < a.hp; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    const seg::SplitPrices<T> pr{(const T*)lprice, (const T*)a.rho, a.hp};
    seg::process_tiles<T, J, 3>(a, blockIdx.x, tiles, gridDim.x, bins, pr, zacc);

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Slot-major kernel: the per-segment step over the slot-major copy (one
// contiguous 256-byte read per slot and array for a whole wave).
template <typename T, int J, bool ALL, bool LDSP, bool TOUCH = false, typename IdxT = int32_t>
__global__ void __launch_bounds__(kSegThreads) k_segments_slots(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.n] prices if LDSP
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    if (LDSP)
        for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    const seg::FlatPrices<T> pr{LDSP ? (const T*)lprice : (const T*)a.rho};
    seg::process_tiles_slots<T, J, ALL, seg::FlatPrices<T>, TOUCH, IdxT>(a, blockIdx.x, tiles,
                                                                       gridDim.x, bins, pr, zacc);

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Slot-major kernel with split prices (head [0, a.hp) in LDS, the rest from
// global memory), for instances whose prices do not fit in LDS.
template <typename T, int J>
__global__ void __launch_bounds__(kSegThreads) k_segments_slots_split(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.hp] prices
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    for (int j = threadIdx.x; j < a.hp; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    const seg::SplitPrices<T> pr{(const T*)lprice, (const T*)a.rho, a.hp};
    seg::process_tiles_slots<T, J, false, seg::SplitPrices<T>>(a, blockIdx.x, tiles, gridDim.x,
                                                              bins, pr, zacc);

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Quad-layout kernel (4-lane groups, 16 rows per wave) over the slot-major
// copy in quad layout; prices all in LDS, or split (head [0, a.hp) in LDS).
template <typename T, int J, typename IdxT, bool SPLIT>
__global__ void __launch_bounds__(kSegThreads) k_segments_quad(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then the LDS prices
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    const int64_t np = SPLIT ? (int64_t)a.hp : a.n;
    for (int64_t j = threadIdx.x; j < np; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + seg::kQuadTileRows - 1) / seg::kQuadTileRows;
    if (SPLIT) {
        const seg::SplitPrices<T> pr{(const T*)lprice, (const T*)a.rho, a.hp};
        seg::process_tiles_quad<T, J, seg::SplitPrices<T>, IdxT>(a, blockIdx.x, tiles, gridDim.x,
                                                                 bins, pr, zacc);
    } else {
        const seg::FlatPrices<T> pr{(const T*)lprice};
        seg::process_tiles_quad<T, J, seg::FlatPrices<T>, IdxT>(a, blockIdx.x, tiles, gridDim.x,
                                                                bins, pr, zacc);
    }

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Mixed kernel: positions [0, P) (rows of at most 32 entries) in the quad
// layout, solved by 4-lane groups (args a, L = P), then positions [P, L) in
// the 8-lane slot-major layout (args b: the same instance viewed from P).
// One launch: the blocks share the LDS prices and bins over both parts.
template <typename T, typename IdxT>
__global__ void __launch_bounds__(kSegThreads) k_segments_mixed(SegArgs a, SegArgs b)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.n] prices
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const seg::FlatPrices<T> pr{(const T*)lprice};
    const int64_t ta = (a.L + seg::kQuadTileRows - 1) / seg::kQuadTileRows;
    seg::process_tiles_quad<T, 8, seg::FlatPrices<T>, IdxT>(a, blockIdx.x, ta, gridDim.x, bins, pr,
                                                            zacc);
    const int64_t tb = (b.L + kSegsPerTile - 1) / kSegsPerTile;
    seg::process_tiles_slots<T, 7, false, seg::FlatPrices<T>, false, IdxT>(b, blockIdx.x, tb,
                                                                          gridDim.x, bins, pr,
                                                                          zacc);

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

// Three-part mixed kernel: positions [0, P2) (rows of at most 16 entries) in
// the pair layout, solved by 2-lane groups (args a2), [P2, P4) (rows of at
// most 32) in the quad layout by 4-lane groups (a4), the rest in the 8-lane
// layout (a8); each view starts at its first position.
// SPLIT: prices [0, a2.hp) in LDS, the rest from global memory.
template <typename T, typename IdxT, bool SPLIT = false>
__global__ void __launch_bounds__(kSegThreads) k_segments_mixed3(SegArgs a2, SegArgs a4, SegArgs a8)
{
    extern __shared__ unsigned long long bins[];   // [a2.H], then the LDS prices
    __shared__ double zsh[kSegThreads / 64];
    const int H = a2.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    const int64_t np = SPLIT ? (int64_t)a2.hp : a2.n;
    for (int64_t j = threadIdx.x; j < np; j += kSegThreads) lprice[j] = ((const T*)a2.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    using PR = typename std::conditional<SPLIT, seg::SplitPrices<T>, seg::FlatPrices<T>>::type;
    PR pr;
    if constexpr (SPLIT)
        pr = PR{(const T*)lprice, (const T*)a2.rho, a2.hp};
    else
        pr = PR{(const T*)lprice};
    const int64_t t2 = (a2.L + seg::kPairTileRows - 1) / seg::kPairTileRows;
    seg::process_tiles_pair<T, 8, PR, IdxT>(a2, blockIdx.x, t2, gridDim.x, bins, pr, zacc);
    const int64_t t4 = (a4.L + seg::kQuadTileRows - 1) / seg::kQuadTileRows;
    seg::process_tiles_quad<T, 8, PR, IdxT>(a4, blockIdx.x, t4, gridDim.x, bins, pr, zacc);
    const int64_t t8 = (a8.L + kSegsPerTile - 1) / kSegsPerTile;
    seg::process_tiles_slots<T, 7, false, PR, false, IdxT>(a8, blockIdx.x, t8, gridDim.x, bins, pr,
                                                         zacc);

    __syncthreads();
    flush_bins(a2, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a2.zpart[blockIdx.x] = z;
    }
}

// Size-class kernel: block b solves tiles [blk[b][1], blk[b][2]) with
// blk[b][0] register slots per lane.  The layout is sorted by row length, so
// a run of tiles has one slot count, and loading every slot of it wastes no
// more than the rounding of the longest row to a multiple of 8.
template <typename T, bool LDSP>
__global__ void __launch_bounds__(kSegThreads) k_segments_cls(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H], then [a.n] prices if LDSP
    __shared__ double zsh[kSegThreads / 64];
    const int H = a.H;
    T* lprice = (T*)(bins + H);
    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    if (LDSP)
        for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
    __syncthreads();

    double zacc = 0.0;
    const int64_t* e = a.blk + 3 * (size_t)blockIdx.x;
    const int J = (int)e[0];
    const int64_t t0 = e[1], t1 = e[2];
    const seg::FlatPrices<T> pr{LDSP ? (const T*)lprice : (const T*)a.rho};
    // FP64 holds at most 4 slots in registers, FP32 7 (longer rows stream
    // the rest from memory in each round)
    switch (J) {
    case 1: seg::process_tiles<T, 1, 3>(a, t0, t1, 1, bins, pr, zacc); break;
    case 2: seg::process_tiles<T, 2, 3>(a, t0, t1, 1, bins, pr, zacc); break;
    case 3: seg::process_tiles<T, 3, 3>(a, t0, t1, 1, bins, pr, zacc); break;
    case 4: seg::process_tiles<T, 4, 3>(a, t0, t1, 1, bins, pr, zacc); break;
    case 5:
        if (sizeof(T) == 4) seg::process_tiles<T, sizeof(T) == 4 ? 5 : 4, 3>(a, t0, t1, 1, bins, pr, zacc);
        break;
    case 6:
        if (sizeof(T) == 4) seg::process_tiles<T, sizeof(T) == 4 ? 6 : 4, 3>(a, t0, t1, 1, bins, pr, zacc);
        break;
    default:
        if (sizeof(T) == 4) seg::process_tiles<T, sizeof(T) == 4 ? 7 : 4, 3>(a, t0, t1, 1, bins, pr, zacc);
        break;
    }

    __syncthreads();
    flush_bins(a, bins);
    for (int o = 32; o > 0; o >>= 1) zacc += __shfl_down(zacc, o, 64);
    if ((threadIdx.x & 63) == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double z = zsh[0];
        for (int q = 1; q < kSegThreads / 64; ++q) z += zsh[q];
        a.zpart[blockIdx.x] = z;
    }
}

}  // namespace

// Segment-kernel variants: (products per lane in registers, pipeline depth).
template <typename T>
struct SegVariant {
    static const void* fn(int variant);
};

template <typename T>
const void* SegVariant<T>::fn(int variant)
{
    switch (variant) {
    case 0: return (const void*)k_segments<T, 8, 1, false>;
    case 1: return (const void*)k_segments<T, 6, 2, false>;
    case 2: return (const void*)k_segments<T, 4, 2, false>;
    case 3: return (const void*)k_segments<T, 8, 2, false>;
    case 5: return (const void*)k_segments<T, 8, 0, false>;
    case 6: return (const void*)k_segments<T, 7, 1, false>;
    case 7: return (const void*)k_segments<T, 7, 3, false>;
    case 8: return (const void*)k_segments<T, 8, 3, false>;
    case 9: return (const void*)k_segments<T, 4, 3, false>;
    case 10: return (const void*)k_segments<T, 7, 1, true>;
    case 11: return (const void*)k_segments<T, 8, 1, true>;
    case 12: return (const void*)k_segments<T, 4, 1, true>;
    case 13: return (const void*)k_segments<T, 7, 3, true>;
    case 14: return (const void*)k_segments<T, 6, 1, true>;
    case 15: return (const void*)k_segments<T, 7, 4, true>;
    case 16: return (const void*)k_segments<T, 8, 4, true>;
    case kSegClassLds: return (const void*)k_segments_cls<T, true>;
    case kSegClassGlobal: return (const void*)k_segments_cls<T, false>;
    case kSegSplit: return (const void*)k_segments_split<T, 7>;
    case kSegSlots: return (const void*)k_segments_slots<T, 7, true, true>;
    case kSegSlots + 1: return (const void*)k_segments_slots<T, 7, false, true>;
    case kSegSlots + 2: return (const void*)k_segments_slots<T, 8, true, true>;
    case kSegSlots + 3: return (const void*)k_segments_slots<T, 4, true, false>;
    case kSegSlots + 4: return (const void*)k_segments_slots<T, 7, false, true, true>;
    case kSegSlots + 5: return (const void*)k_segments_slots<T, 4, false, false, true>;
    case kSegSlotsSplit: return (const void*)k_segments_slots_split<T, 7>;
    case kSegSlotsSplit + 1: return (const void*)k_segments_slots_split<T, 4>;
    case kSegSlotsJ4: return (const void*)k_segments_slots<T, 4, false, true>;
    case kSegSlots16: return (const void*)k_segments_slots<T, 7, false, true, false, uint16_t>;
    case kSegSlots16 + 1: return (const void*)k_segments_slots<T, 4, false, true, false, uint16_t>;
    case kSegSlots16 + 2: return (const void*)k_segments_slots<T, 4, true, false, false, uint16_t>;
    case kSegQuad: return (const void*)k_segments_quad<T, 8, uint16_t, false>;
    case kSegQuad + 1: return (const void*)k_segments_quad<T, 8, int32_t, true>;
    case kSegQuad + 2: return (const void*)k_segments_quad<T, 8, int32_t, false>;
    case kSegMixed: return (const void*)k_segments_mixed<T, uint16_t>;
    case kSegMixed + 1: return (const void*)k_segments_mixed<T, int32_t>;
    case kSegMixed3: return (const void*)k_segments_mixed3<T, uint16_t>;
    case kSegMixed3 + 1: return (const void*)k_segments_mixed3<T, int32_t>;
    case kSegMixed3 + 2: return (const void*)k_segments_mixed3<T, int32_t, true>;
    case kSegMixed3 + 3: return (const void*)k_segments_mixed3<T, uint16_t, true>;
    default: return (const void*)k_segments<T, 4, 1, false>;
    }
}

template <typename T>
hipError_t launch_segments_mixed(const SegArgs& a, const SegArgs& b, int grid, int variant,
                                 hipStream_t s)
{
    const size_t lds = seg_lds_bytes(a.H, a.n, sizeof(T), variant);
    void* args[] = {(void*)&a, (void*)&b};
    return hipLaunchKernel(SegVariant<T>::fn(variant), dim3(grid), dim3(kSegThreads), args, lds,
                           s);
}

template <typename T>
hipError_t launch_segments_mixed3(const SegArgs& a2, const SegArgs& a4, const SegArgs& a8, int grid,
                                  int variant, hipStream_t s)
{
    const size_t lds = seg_lds_bytes(a2.H, seg_split(variant) ? a2.hp : a2.n, sizeof(T), variant);
    void* args[] = {(void*)&a2, (void*)&a4, (void*)&a8};
    return hipLaunchKernel(SegVariant<T>::fn(variant), dim3(grid), dim3(kSegThreads), args, lds,
                           s);
}

template <typename T>
hipError_t launch_segments(const SegArgs& a, int grid, int variant, hipStream_t s)
{
    const size_t lds = seg_lds_bytes(a.H, seg_split(variant) ? a.hp : a.n, sizeof(T), variant);
    void* args[] = {(void*)&a};
    return hipLaunchKernel(SegVariant<T>::fn(variant), dim3(grid), dim3(kSegThreads), args, lds,
                           s);
}

template <typename T>
int segment_blocks_per_cu(int H, int64_t n, int variant)   // n: prices held in LDS
{
    int blocks = 0;
    const size_t lds = seg_lds_bytes(H, n, sizeof(T), variant);
    const void* f = SegVariant<T>::fn(variant);
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, f, kSegThreads, lds) != hipSuccess)
        return 1;
    return blocks < 1 ? 1 : blocks;
}

template hipError_t launch_segments<float>(const SegArgs&, int, int, hipStream_t);
template hipError_t launch_segments_mixed<float>(const SegArgs&, const SegArgs&, int, int,
                                                 hipStream_t);
template hipError_t launch_segments_mixed<double>(const SegArgs&, const SegArgs&, int, int,
                                                  hipStream_t);
template hipError_t launch_segments_mixed3<float>(const SegArgs&, const SegArgs&, const SegArgs&, int,
                                                  int, hipStream_t);
template hipError_t launch_segments_mixed3<double>(const SegArgs&, const SegArgs&, const SegArgs&,
                                                   int, int, hipStream_t);
template hipError_t launch_segments<double>(const SegArgs&, int, int, hipStream_t);
template int segment_blocks_per_cu<float>(int, int64_t, int);
template int segment_blocks_per_cu<double>(int, int64_t, int);

}  // namespace cblp

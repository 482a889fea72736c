// Single-instance segment kernel: the per-segment primal step over every
// segment and the per-block LDS-bin rows of product sales (device code in
// segment_core.hpp).
#include "segment_core.hpp"

namespace cblp {
namespace {

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
    seg::process_tiles<T, J, DEPTH>(a, blockIdx.x, tiles, gridDim.x, bins,
                                    LDSP ? (const T*)lprice : (const T*)a.rho, zacc);

    __syncthreads();
    unsigned long long* out = a.part_S + (size_t)blockIdx.x * (size_t)H;
    for (int j = threadIdx.x; j < H; j += kSegThreads) out[j] = bins[j];

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
    default: return (const void*)k_segments<T, 4, 1, false>;
    }
}

template <typename T>
hipError_t launch_segments(const SegArgs& a, int grid, int variant, hipStream_t s)
{
    const size_t lds = seg_lds_bytes(a.H, a.n, sizeof(T), variant);
    void* args[] = {(void*)&a};
    return hipLaunchKernel(SegVariant<T>::fn(variant), dim3(grid), dim3(kSegThreads), args, lds,
                           s);
}

template <typename T>
int segment_blocks_per_cu(int H, int64_t n, int variant)
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
template hipError_t launch_segments<double>(const SegArgs&, int, int, hipStream_t);
template int segment_blocks_per_cu<float>(int, int64_t, int);
template int segment_blocks_per_cu<double>(int, int64_t, int);

}  // namespace cblp

// Per-segment primal step and deterministic sales scatter.
//
// The inner problem of one segment (Section 4.1, in its GAM form): with
// vt0 = v0 + sum_{N_l} w and vt_j = v_j - w_j > 0, offering S earns
// R(S) = sum_S rho_j v_j / (vt0 + sum_S vt_j) per arrival; the best
// response is R* = max(0, max_S R(S)) on S* = {j : rho_j v_j > R* vt_j}
// (a prefix of the products ordered by rho_j v_j / vt_j, the nested family
// of Section 4.4).  R* comes from Dinkelbach's parametric iteration: from
// R = 0 take S(R) = {rho_j v_j > R vt_j} and set R <- R(S(R)) until S(R)
// stops changing.  R never decreases, so the sets shrink monotonically and
// the loop ends after at most |N_l| + 1 rounds (2-4 in practice).  No sort
// and no per-product division is needed; every round is one compare and
// two adds per product plus one 16-lane reduction.
//
// Sales s_lj = lambda_l v_lj / (vt0 + sum_{S*} vt) are rounded once to
// 64-bit fixed point (scale 2^bits, bits chosen so that sum_l lambda_l fits)
// and summed with integer atomics, so the totals do not depend on the order
// of the additions.  Products [0, H) - the popular head when products are
// numbered by popularity - accumulate in LDS bins of each block and are
// written out as one partial row per block; the rest go to global atomics.
#include "common.hpp"

namespace cblp {
namespace {

template <typename X>
__device__ __forceinline__ X group_sum(X x)
{
    x += __shfl_xor(x, 8, kGroup);
    x += __shfl_xor(x, 4, kGroup);
    x += __shfl_xor(x, 2, kGroup);
    x += __shfl_xor(x, 1, kGroup);
    return x;
}

// Software pipeline over the tiles a block visits: the row bounds of tile
// i+3, the CSR entries of tile i+2 and the price gathers of tile i+1 are in
// flight while tile i is solved, so each wave keeps several independent
// memory round trips outstanding instead of one dependent chain per tile.
template <typename T>
struct Bounds {
    int64_t b;
    int k;
    T vt0, lam;
};

template <typename T>
struct Raw {          // CSR entries of one segment held by this lane
    int32_t id[kJ];
    T v[kJ], w[kJ];
};

template <typename T>
struct Cooked {       // rho v, v - w, v and product id per slot
    T num[kJ], den[kJ], vv[kJ];
    int32_t id[kJ];
};

template <typename T>
__device__ __forceinline__ Bounds<T> load_bounds(const SegArgs& a, int64_t l)
{
    Bounds<T> B;
    B.b = 0;
    B.k = 0;
    B.vt0 = T(1);
    B.lam = T(0);
    if (l < a.L) {
        B.b = a.seg_ptr[l];
        B.k = (int)(a.seg_ptr[l + 1] - B.b);
        B.vt0 = ((const T*)a.vt0)[l];
        B.lam = ((const T*)a.lam)[l];
    }
    return B;
}

template <typename T>
__device__ __forceinline__ Raw<T> load_raw(const SegArgs& a, const Bounds<T>& B, int g)
{
    Raw<T> R;
#pragma unroll
    for (int s = 0; s < kJ; ++s) {
        const int q = g + kGroup * s;
        if (q < B.k) {
            R.id[s] = a.idx[B.b + q];
            R.v[s] = ((const T*)a.v)[B.b + q];
            R.w[s] = ((const T*)a.w)[B.b + q];
        } else {
            R.id[s] = -1;
            R.v[s] = T(0);
            R.w[s] = T(0);
        }
    }
    return R;
}

template <typename T>
__device__ __forceinline__ Cooked<T> cook(const SegArgs& a, const Raw<T>& R)
{
    Cooked<T> C;
    const T* rho = (const T*)a.rho;
#pragma unroll
    for (int s = 0; s < kJ; ++s) {
        if (R.id[s] >= 0) {
            C.id[s] = R.id[s];
            C.vv[s] = R.v[s];
            C.den[s] = R.v[s] - R.w[s];
            C.num[s] = rho[R.id[s]] * R.v[s];
        } else {
            C.id[s] = 0;
            C.vv[s] = T(0);
            C.den[s] = T(1);
            C.num[s] = T(0);   // never offered: 0 > R * 1 fails for R >= 0
        }
    }
    return C;
}

template <typename T>
__global__ void __launch_bounds__(kSegThreads) k_segments(SegArgs a)
{
    extern __shared__ unsigned long long bins[];   // [a.H]
    __shared__ double zsh[kSegThreads / 64];
    const T* __restrict__ v = (const T*)a.v;
    const T* __restrict__ w = (const T*)a.w;
    const T* __restrict__ rho = (const T*)a.rho;
    const int32_t* __restrict__ idx = a.idx;
    const int H = a.H;
    const int g = threadIdx.x & (kGroup - 1);
    const int grp = threadIdx.x / kGroup;

    for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
    __syncthreads();

    double zacc = 0.0;
    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    const int64_t stride = gridDim.x;
    int64_t tile = blockIdx.x;
    auto seg_of = [&](int64_t t) { return t * kSegsPerTile + grp; };

    // prologue: fill the pipeline
    Bounds<T> Bc = load_bounds<T>(a, seg_of(tile));
    Bounds<T> B1 = load_bounds<T>(a, seg_of(tile + stride));
    Raw<T> R1 = load_raw<T>(a, B1, g);
    Bounds<T> B2 = load_bounds<T>(a, seg_of(tile + 2 * stride));
    Cooked<T> Cc = cook<T>(a, load_raw<T>(a, Bc, g));

    for (; tile < tiles; tile += stride) {
        // issue the next stages before touching the current tile
        Raw<T> R2 = load_raw<T>(a, B2, g);
        Bounds<T> B3 = load_bounds<T>(a, seg_of(tile + 3 * stride));
        Cooked<T> C1 = cook<T>(a, R1);

        const int64_t l = seg_of(tile);
        const int64_t b = Bc.b;
        const int k = Bc.k;
        const T vt0 = Bc.vt0;
        auto sums = [&](T R, T& N, T& Dn, int& cnt) {
            T n_ = T(0), d_ = T(0);
            int c_ = 0;
#pragma unroll
            for (int s = 0; s < kJ; ++s) {
                if (Cc.num[s] > R * Cc.den[s]) {
                    n_ += Cc.num[s];
                    d_ += Cc.den[s];
                    ++c_;
                }
            }
            for (int q = kGroup * kJ + g; q < k; q += kGroup) {
                const T x = v[b + q];
                const T nn = rho[idx[b + q]] * x;
                const T dd = x - w[b + q];
                if (nn > R * dd) {
                    n_ += nn;
                    d_ += dd;
                    ++c_;
                }
            }
            N = group_sum(n_);
            Dn = group_sum(d_);
            cnt = group_sum(c_);
        };
        // Dinkelbach: R defines the set whose sums are (N, Dn, cnt)
        T R = T(0), N, Dn;
        int cnt;
        sums(R, N, Dn, cnt);
        for (int round = 0; round < k + 2; ++round) {
            const T Rn = cnt > 0 ? N / (vt0 + Dn) : T(0);
            T N2, D2;
            int c2;
            sums(Rn, N2, D2, c2);
            if (c2 == cnt) break;   // nested sets of equal size are equal
            R = Rn;
            N = N2;
            Dn = D2;
            cnt = c2;
        }
        const T Rstar = cnt > 0 ? N / (vt0 + Dn) : T(0);
        const T Dl = vt0 + Dn;
        const T lam = Bc.lam;
#pragma unroll
        for (int s = 0; s < kJ; ++s) {
            if (Cc.num[s] > R * Cc.den[s]) {
                const T sj = lam * Cc.vv[s] / Dl;
                const unsigned long long q =
                    (unsigned long long)__double2ll_rn((double)sj * a.fx_scale);
                if (Cc.id[s] < H)
                    atomicAdd(&bins[Cc.id[s]], q);
                else
                    atomicAdd(&a.S_fx[Cc.id[s]], q);
            }
        }
        for (int q = kGroup * kJ + g; q < k; q += kGroup) {
            const T x = v[b + q];
            const int32_t j = idx[b + q];
            if (rho[j] * x > R * (x - w[b + q])) {
                const T sj = lam * x / Dl;
                const unsigned long long qq =
                    (unsigned long long)__double2ll_rn((double)sj * a.fx_scale);
                if (j < H)
                    atomicAdd(&bins[j], qq);
                else
                    atomicAdd(&a.S_fx[j], qq);
            }
        }
        if (g == 0 && l < a.L) {
            zacc += (double)lam * (double)Rstar;
            if (a.seg_R) ((T*)a.seg_R)[l] = Rstar;
        }
        // rotate the pipeline
        Bc = B1;
        Cc = C1;
        B1 = B2;
        R1 = R2;
        B2 = B3;
    }
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

template <typename T>
hipError_t launch_segments(const SegArgs& a, int grid, hipStream_t s)
{
    const size_t lds = (size_t)a.H * sizeof(unsigned long long);
    hipLaunchKernelGGL(k_segments<T>, dim3(grid), dim3(kSegThreads), lds, s, a);
    return hipGetLastError();
}

template <typename T>
int segment_blocks_per_cu(int H)
{
    int blocks = 0;
    const size_t lds = (size_t)H * sizeof(unsigned long long);
    (void)hipFuncSetAttribute((const void*)k_segments<T>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_segments<T>, kSegThreads, lds) !=
        hipSuccess)
        return 1;
    return blocks < 1 ? 1 : blocks;
}

template hipError_t launch_segments<float>(const SegArgs&, int, hipStream_t);
template hipError_t launch_segments<double>(const SegArgs&, int, hipStream_t);
template int segment_blocks_per_cu<float>(int);
template int segment_blocks_per_cu<double>(int);

}  // namespace cblp

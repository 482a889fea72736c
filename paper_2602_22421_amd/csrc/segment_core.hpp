// Device code of the per-segment primal step, shared by the single-instance
// and the batched segment kernels.
//
// The inner problem of one segment (Section 4.1, in its GAM form): with
// vt0 = v0 + sum_{N_l} w and vt_j = v_j - w_j > 0, offering S earns
// R(S) = sum_S rho_j v_j / (vt0 + sum_S vt_j) per arrival; the best
// response is R* = max(0, max_S R(S)) on S* = {j : rho_j v_j > R* vt_j}
// (a prefix of the products ordered by rho_j v_j / vt_j, the nested family
// of Section 4.4).  R* comes from Dinkelbach's parametric iteration: from a
// start R0 >= 0 take S(R) = {rho_j v_j > R vt_j} and set R <- R(S(R)) until
// S(R) stops changing.  After the first step R <= R* and R never decreases,
// so the sets are nested and the loop ends after at most |N_l| + 1 rounds.
// The start is the segment's R* of the previous call (0 at creation): the
// duals move little between iterations, so most segments finish in two
// rounds.  Each round is one compare and two masked adds per product and
// three 8-lane DPP reductions; no sort and no per-product division.
//
// Sales s_lj = (lambda_l / D_l) v_lj with D_l = vt0 + sum_{S*} vt are rounded
// once to fixed point (scale 2^bits: FP32 rounds to 32-bit quanta, FP64 to
// 64-bit ones) and summed as 64-bit integers, so the totals do not depend on
// the order of the additions.  Products [0, H) - the popular head when
// products are numbered by popularity - accumulate in LDS bins of each block
// (64-bit for the first H64, 32-bit for the rest, sized so that no 32-bit
// sum can wrap) and leave LDS at the block's end; the rest use global atomics.
//
// Layout: an 8-lane group owns one segment of the library's size-sorted
// copy; lane g holds products g, g+8, ..., g+56 of the row in registers and
// re-reads products past 64 from memory in each round.  A block of 1024
// threads holds 128 groups and strides over tiles of 128 consecutive
// positions; the slot loops run to the longest row of the wave, which the
// size sort keeps close to every row's own length.  Row bounds of tile i+3,
// CSR entries of tile i+2 and price gathers of tile i+1 are in flight while
// tile i is solved.
#pragma once

#include "common.hpp"

namespace cblp {
namespace seg {

// Every product and sum below is rounded as written (no contraction into
// fused multiply-adds except the explicit ones), so all kernel variants - and
// register slots and streamed slots within one - give the same bits.
#pragma clang fp contract(off)

// 8-lane sum with DPP inside half rows: mirror, then swap pairs, then swap
// neighbours.  Every lane of the group ends with the same bits: each step
// adds two values that the other lane of the pair adds in the opposite
// order, and floating-point addition is commutative.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
constexpr int kHalfMirror = 0x141, kQuadSwap2 = 0x4E, kQuadSwap1 = 0xB1;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_i<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_move(int x)
{
    return dpp_i<CTRL>(x);
}

template <typename X>
__device__ __forceinline__ X group_sum(X x)
{
    x += dpp_move<kHalfMirror>(x);
    x += dpp_move<kQuadSwap2>(x);
    x += dpp_move<kQuadSwap1>(x);
    return x;
}

// Pipeline stages.  They are branch-free and do no arithmetic on loaded
// values, so a wait for a load is emitted only where the value is used, one
// pipeline step later.  Slots past a row's end load entry 0 of the arrays
// (never used; the host passes a one-element buffer for an empty instance).
template <typename T>
struct Bounds {
    int64_t b, e;     // row [b, e) of the sorted layout
    T vt0, lam, R0;
    bool live;        // a segment of the instance (not past its end)
};

template <typename T, int J>
struct Raw {          // CSR entries of one row held by this lane
    int32_t id[J];
    T v[J], den[J];
};

template <typename T>
__device__ __forceinline__ Bounds<T> load_bounds(const SegArgs& a, int64_t p)
{
    const int64_t pc = p < a.L ? p : 0;
    Bounds<T> B;
    B.b = a.ptr[pc];
    B.e = a.ptr[pc + 1];
    B.vt0 = ((const T*)a.vt0)[pc];
    B.lam = ((const T*)a.lam)[pc];
    B.R0 = ((const T*)a.Rwarm)[pc];
    B.live = p < a.L;
    return B;
}

// Row length, taken where it is used (a pipeline step after the load).  The
// 64-bit compare keeps both halves of e live, so the compiler never reuses a
// register that a row bound is still being loaded into, which would force a
// wait for every load in flight.
template <typename T>
__device__ __forceinline__ int row_len(const Bounds<T>& B)
{
    return (B.live && B.e > B.b) ? (int)(B.e - B.b) : 0;
}

// The library pads its CSR copy with kGroup * kMaxJ entries, so slot s of
// every lane reads base + 8 s with an immediate offset; slots past a row's
// end read the next row (masked off when used).  ALL: every one of the J
// slots is loaded, so the number of loads in flight is fixed and the waits
// for them can count exactly; otherwise only the first jw slots - the
// longest row of the wave - are loaded.
template <typename T, int J, bool ALL>
__device__ __forceinline__ Raw<T, J> load_raw(const SegArgs& a, const Bounds<T>& B, int g, int jw)
{
    Raw<T, J> R;
    const int32_t* pi = a.idx + B.b + g;
    const T* pv = (const T*)a.v + B.b + g;
    const T* pd = (const T*)a.den + B.b + g;
#pragma unroll
    for (int s = 0; s < J; ++s) {
        if (ALL || s < jw) {
            R.id[s] = pi[kGroup * s];
            R.v[s] = pv[kGroup * s];
            R.den[s] = pd[kGroup * s];
        } else {
            R.id[s] = 0;
            R.v[s] = T(0);
            R.den[s] = T(1);
        }
    }
    return R;
}

// Price tables: all in one memory (global or an LDS copy), or split with
// the popular head [0, hp) in LDS and the rest read from global memory.
template <typename T>
struct FlatPrices {
    const T* __restrict__ p;
    __device__ __forceinline__ T operator[](int j) const { return p[j]; }
};
template <typename T>
struct SplitPrices {
    const T* __restrict__ lds;
    const T* __restrict__ glob;
    int hp;
    // both reads for every lane (no pointer select, which would make a flat
    // access); head lanes read global entry 0, one shared cache line
    __device__ __forceinline__ T operator[](int j) const
    {
        const bool head = j < hp;
        const T l = lds[head ? j : 0];
        const T g = glob[head ? 0 : j];
        return head ? l : g;
    }
};

template <typename T, int J, bool ALL, typename PR>
__device__ __forceinline__ void gather(const PR& prices, const Raw<T, J>& R, T (&p)[J], int jw)
{
#pragma unroll
    for (int s = 0; s < J; ++s) p[s] = (ALL || s < jw) ? prices[R.id[s]] : T(0);
}

// wave-uniform slot count: ceil(k / 8) of the longest row among the wave's
// eight groups (not capped at J: it also bounds the Dinkelbach rounds)
// (the first lane of each group holds the group's value; eight lane reads
// into scalar registers avoid the round trips of cross-lane shuffles)
template <int J>
__device__ __forceinline__ int wave_slots(int k)
{
    const int jw = (k + kGroup - 1) / kGroup;
    int m = __builtin_amdgcn_readlane(jw, 0);
#pragma unroll
    for (int q = 1; q < 64 / kGroup; ++q) m = max(m, __builtin_amdgcn_readlane(jw, q * kGroup));
    return m;
}

// R = N / D.  FP32 uses the hardware reciprocal (about one ulp); the value
// only sets the next threshold and R*, both well inside the FP32 tolerance.
__device__ __forceinline__ float ratio(float n, float d) { return n * __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double ratio(double n, double d) { return n / d; }

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Fixed-point quantum of a sale lambda v / D, given ls = (lambda / D) 2^bits
// (a power-of-two scaling, exact).  FP32: the quantum is below 2^30; round
// half up by truncating ls v + 1/2.  FP64: round to nearest.
__device__ __forceinline__ unsigned long long quantum(float ls, float v)
{
    return (unsigned long long)(unsigned)(int)__builtin_fmaf(ls, v, 0.5f);
}
__device__ __forceinline__ unsigned long long quantum(double ls, double v)
{
    return (unsigned long long)__double2ll_rn(ls * v);
}

// One sale of q quanta of product j.  Products [0, a.H64) are summed in the
// block's 64-bit LDS bins, [a.H64, a.H) in the 32-bit LDS bins that follow
// them, the rest straight in the global 64-bit sums.  A product gets a
// 32-bit bin only when a bound on its sales within every block (each sale
// at most lambda v / (vt0 + v - w), whatever the assortment) stays below
// 2^32 quanta, so the 32-bit sums never wrap (the host checks the bound;
// FP64 handles keep H64 = H).
template <typename T>
__device__ __forceinline__ void add_sale(const SegArgs& a, unsigned long long* bins, int j,
                                         unsigned long long q)
{
    if (j < a.H64)
        atomicAdd(&bins[j], q);
    else if (sizeof(T) == 4 && j < a.H)
        atomicAdd((unsigned*)(bins + a.H64) + (j - a.H64), (unsigned)q);
    else
        atomicAdd(&a.S_fx[j], q);
}

// J: products per lane held in registers (rows longer than 8 J stream the
// rest).  DEPTH 1 keeps the CSR entries of the next tile (and the row bounds
// of the one after) in flight while a tile is solved; DEPTH 0 none; DEPTH 2
// one more tile of entries and the price gathers.  DEPTH 3 is DEPTH 1 with
// every slot loaded and the loads of an iteration issued in the order they
// are consumed (this tile's price gathers, the next tile's entries, the
// bounds of the tile after), so the solve waits for its gathers alone; DEPTH
// 4 is the same order with only the wave's jw slots loaded.  The
// block visits tiles tile, tile + stride, ... below `tiles`; sales go to the
// LDS bins (products < a.H) or the global tail; lambda R* is added to zacc (fixed
// point).
//
// prices: the reduced revenues rho_j as a FlatPrices (a.rho itself or a copy
// of it in LDS; the compiler sees which memory it is) or a SplitPrices.
template <typename T, int J, int DEPTH, typename PR>
__device__ __forceinline__ void process_tiles(const SegArgs& a, int64_t tile, int64_t tiles,
                                              int64_t stride, unsigned long long* bins,
                                              const PR& prices, ZAcc& zacc)
{
    constexpr bool ALL = DEPTH == 3;
    constexpr bool ORDERED = DEPTH >= 3;   // DEPTH 4: ordered issue, only jw slots loaded
    const T* __restrict__ vg = (const T*)a.v;
    const T* __restrict__ dg = (const T*)a.den;
    const PR& rho = prices;
    const int32_t* __restrict__ idx = a.idx;
    const int g = threadIdx.x & (kGroup - 1);
    const int grp = threadIdx.x / kGroup;
    auto pos_of = [&](int64_t t) { return t * kSegsPerTile + grp; };

    if (tile < tiles) {
        Bounds<T> Bc = load_bounds<T>(a, pos_of(tile));
        int jc = wave_slots<J>(row_len(Bc));
        Raw<T, J> Rc = load_raw<T, J, ALL>(a, Bc, g, jc);
        T Pc[J];
        if (DEPTH == 2) gather<T, J, ALL, PR>(rho, Rc, Pc, jc);
        Bounds<T> B1 = load_bounds<T>(a, pos_of(tile + stride));
        int j1 = 0;
        Raw<T, J> R1;
        if (DEPTH == 2) {
            j1 = wave_slots<J>(row_len(B1));
            R1 = load_raw<T, J, ALL>(a, B1, g, j1);
        }
        Bounds<T> B2;
        if (!ORDERED) B2 = load_bounds<T>(a, pos_of(tile + 2 * stride));

        for (; tile < tiles; tile += stride) {
            // issue the next stages before touching the current tile
            Raw<T, J> R2;
            Bounds<T> B3;
            T P1[J];
            int j2 = 0;
            if (ORDERED) {
                gather<T, J, ALL, PR>(rho, Rc, Pc, jc);
                // keep the gathers ahead of the next tile's loads: a wait for
                // a gather then never waits for those loads
                __builtin_amdgcn_sched_barrier(0);
                j1 = wave_slots<J>(row_len(B1));
                R1 = load_raw<T, J, ALL>(a, B1, g, j1);
                B2 = load_bounds<T>(a, pos_of(tile + 2 * stride));
            } else if (DEPTH == 2) {
                j2 = wave_slots<J>(row_len(B2));
                R2 = load_raw<T, J, ALL>(a, B2, g, j2);
                B3 = load_bounds<T>(a, pos_of(tile + 3 * stride));
                gather<T, J, ALL, PR>(rho, R1, P1, j1);
            } else if (DEPTH == 1) {
                j1 = wave_slots<J>(row_len(B1));
                R1 = load_raw<T, J, ALL>(a, B1, g, j1);
                gather<T, J, ALL, PR>(rho, Rc, Pc, jc);
            } else {
                gather<T, J, ALL, PR>(rho, Rc, Pc, jc);
            }

            const int64_t p = pos_of(tile);
            const int64_t b = Bc.b;
            const int k = row_len(Bc);
            const T vt0 = Bc.vt0;
            const int jw = jc;

            // slots past the row hold num = 0, which never enters a set
            // (0 > R den is false for R >= 0 and den > 0)
            T num[J], den[J];
#pragma unroll
            for (int s = 0; s < J; ++s) {
                const bool ok = g + kGroup * s < k;
                num[s] = ok ? Pc[s] * Rc.v[s] : T(0);
                den[s] = Rc.den[s];
            }
            // Dinkelbach with wave-wide membership masks.  A full pass forms
            // S(R) - one ballot per slot - and its sums; a check pass only
            // compares S(R') with S(R).  A group whose set did not change
            // repeats the same sums, so the loop is uniform over the wave and
            // ends when no group of the wave changes.
            const int js = jw < J ? jw : J;
            unsigned long long mask[J];
            auto full = [&](T R, T& N, T& Dn) {
                T n_ = T(0), d_ = T(0);
#pragma unroll
                for (int s = 0; s < J; ++s) {
                    mask[s] = 0ull;
                    if (s >= js) continue;
                    const bool in = num[s] > R * den[s];
                    mask[s] = __ballot(in);
                    // fma by 0 or 1 adds the value or nothing, rounded once
                    const T w = in ? T(1) : T(0);
                    n_ = fmadd(w, num[s], n_);
                    d_ = fmadd(w, den[s], d_);
                }
                for (int q = kGroup * J + g; q < k; q += kGroup) {
                    const T nn = rho[idx[b + q]] * vg[b + q];
                    const T dd = dg[b + q];
                    const T w = nn > R * dd ? T(1) : T(0);
                    n_ = fmadd(w, nn, n_);
                    d_ = fmadd(w, dd, d_);
                }
                N = group_sum(n_);
                Dn = group_sum(d_);
            };
            auto changed = [&](T R, T Rn) {
                unsigned long long diff = 0ull;
#pragma unroll
                for (int s = 0; s < J; ++s) {
                    if (s >= js) break;
                    diff |= __ballot(num[s] > Rn * den[s]) ^ mask[s];
                }
                if (jw > J) {                     // rows past the register slots
                    bool t = false;
                    for (int q = kGroup * J + g; q < k; q += kGroup) {
                        const T nn = rho[idx[b + q]] * vg[b + q];
                        const T dd = dg[b + q];
                        t = t || ((nn > Rn * dd) != (nn > R * dd));
                    }
                    diff |= __ballot(t);
                }
                return diff;
            };
            // R is the threshold of the current set, (N, Dn) its sums and Rs
            // its ratio; members have num > 0, so the set is empty exactly
            // when N == 0.  In exact arithmetic the ratios rise until the set
            // repeats.  Ties within an ulp can instead make a group alternate
            // between two sets; the loop then runs to its cap, and such a
            // group keeps the set of larger ratio of the two, which does not
            // depend on where the iteration started.
            T R = Bc.R0, N, Dn;
            full(R, N, Dn);
            T Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
            T pR = R, pN = N, pD = Dn, pRs = Rs;
            unsigned long long diff = 0ull;
            for (int round = 0; round <= kGroup * jw + 1; ++round) {
                diff = changed(R, Rs);
                if (diff == 0ull) break;
                pR = R;
                pN = N;
                pD = Dn;
                pRs = Rs;
                R = Rs;
                full(R, N, Dn);
                Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
            }
            if (diff != 0ull) {
                const unsigned long long now = changed(R, Rs);
                const bool cycling = ((now >> (threadIdx.x & 56)) & 0xFFull) != 0ull;
                if (cycling && pRs > Rs) {
                    R = pR;
                    N = pN;
                    Dn = pD;
                    Rs = pRs;
                }
            }
            const T Rstar = Rs;
            const T lamD = ratio(Bc.lam, vt0 + Dn) * (T)a.fx_scale;
#pragma unroll
            for (int s = 0; s < J; ++s) {
                if (s >= js) break;
                if (num[s] > R * den[s]) {
                    const unsigned long long q = quantum(lamD, Rc.v[s]);
                    const int32_t j = Rc.id[s];
                    add_sale<T>(a, bins, j, q);
                }
            }
            for (int q = kGroup * J + g; q < k; q += kGroup) {
                const T x = vg[b + q];
                const int32_t j = idx[b + q];
                if (rho[j] * x > R * dg[b + q]) {
                    const unsigned long long qq = quantum(lamD, x);
                    add_sale<T>(a, bins, j, qq);
                }
            }
            if (g == 0 && p < a.L) {
                zacc.add((double)Bc.lam * (double)Rstar, z_ok((double)Rstar, a.z_rmax), a.z_scale);
                ((T*)a.Rwarm)[p] = Rstar;
                if (a.seg_R) ((T*)a.seg_R)[a.perm[p]] = Rstar;
            }
            // rotate the pipeline
            Bc = B1;
            Rc = R1;
            jc = j1;
            if (ORDERED) {
                B1 = B2;
            } else if (DEPTH == 2) {
#pragma unroll
                for (int s = 0; s < J; ++s) Pc[s] = P1[s];
                B1 = B2;
                R1 = R2;
                j1 = j2;
                B2 = B3;
            } else if (DEPTH == 1) {
                B1 = B2;
                B2 = load_bounds<T>(a, pos_of(tile + 3 * stride));
            } else {
                Bc = load_bounds<T>(a, pos_of(tile + stride));
                jc = wave_slots<J>(row_len(Bc));
                Rc = load_raw<T, J, ALL>(a, Bc, g, jc);
            }
        }
    }
}


// ---------------------------------------------------------------- slot-major
// The same per-segment step over the slot-major copy: a wave owns the eight
// rows of one wave-tile, and slot s of the whole wave is 64 consecutive
// entries (lane 8 q + g holds entry g + 8 s of row q), so every load of a
// slot is one contiguous 256-byte read.  Places past a row's end hold v = 0
// (num = 0 never enters a set), so rows need no length masks; slots past the
// wave-tile's own count (ALL loads J of them) are masked by one scalar test.
template <typename T>
struct WaveBounds {
    int64_t b0, b1;   // entries [b0, b1) of the wave-tile (same in every lane)
    bool wlive;       // the wave-tile exists
    T vt0, lam, R0;
    bool live;        // this group's row exists
};

// Loads only; the slot count is formed where it is used, a pipeline step
// later, so no wait is needed here (woff has one spare entry at the end).
template <typename T>
__device__ __forceinline__ WaveBounds<T> load_wave_bounds(const SegArgs& a, int64_t t, int wv,
                                                         int q)
{
    const int64_t W = (a.L + kGroup - 1) / kGroup;
    const int64_t w = t * (kSegsPerTile / kGroup) + wv;
    const int64_t wc = w < W ? w : 0;
    WaveBounds<T> B;
    B.b0 = a.woff[wc];
    B.b1 = a.woff[wc + 1];
    B.wlive = w < W;
    const int64_t p = w * kGroup + q;
    const int64_t pc = p < a.L ? p : 0;
    B.vt0 = ((const T*)a.vt0)[pc];
    B.lam = ((const T*)a.lam)[pc];
    B.R0 = ((const T*)a.Rwarm)[pc];
    B.live = p < a.L;
    return B;
}

template <typename T>
__device__ __forceinline__ int64_t wave_base(const WaveBounds<T>& B)
{
    return ((int64_t)__builtin_amdgcn_readfirstlane((int)(B.b0 >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)B.b0);
}
template <typename T>
__device__ __forceinline__ int wave_jw(const WaveBounds<T>& B)
{
    return __builtin_amdgcn_readfirstlane(B.wlive ? (int)((B.b1 - B.b0) >> 6) : 0);
}

// IdxT: the slot-major copy's product ids, int32_t or uint16_t (n <= 65536)
template <typename T, int J, bool ALL, typename IdxT = int32_t>
__device__ __forceinline__ Raw<T, J> load_slots(const SegArgs& a, const WaveBounds<T>& B, int lane)
{
    Raw<T, J> R;
    const int64_t base = wave_base(B);
    const int jw = ALL ? J : wave_jw(B);
    const IdxT* pi = (const IdxT*)a.idx3 + base + lane;
    const T* pv = (const T*)a.v3 + base + lane;
    const T* pd = (const T*)a.den3 + base + lane;
#pragma unroll
    for (int s = 0; s < J; ++s) {
        if (ALL || s < jw) {
            R.id[s] = (int32_t)pi[64 * s];
            R.v[s] = pv[64 * s];
            R.den[s] = pd[64 * s];
        } else {
            R.id[s] = 0;
            R.v[s] = T(0);
            R.den[s] = T(1);
        }
    }
    return R;
}

template <typename T, int J, bool ALL, typename PR, typename IdxT = int32_t, bool PSEG = false>
__device__ __forceinline__ void process_tiles_slots(const SegArgs& a, int64_t tile, int64_t tiles,
                                                    int64_t stride, unsigned long long* bins,
                                                    const PR& rho, ZAcc& zacc)
{
    const T* __restrict__ v3 = (const T*)a.v3;
    const T* __restrict__ d3 = (const T*)a.den3;
    const IdxT* __restrict__ i3 = (const IdxT*)a.idx3;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int q = lane / kGroup;
    if (tile >= tiles) return;

    WaveBounds<T> Bc = load_wave_bounds<T>(a, tile, wv, q);
    Raw<T, J> Rc = load_slots<T, J, ALL, IdxT>(a, Bc, lane);
    WaveBounds<T> B1 = load_wave_bounds<T>(a, tile + stride, wv, q);
    WaveBounds<T> B2;
    T Pc[J];
    for (; tile < tiles; tile += stride) {
        gather<T, J, true, PR>(rho, Rc, Pc, J);
        __builtin_amdgcn_sched_barrier(0);
        const Raw<T, J> R1 = load_slots<T, J, ALL, IdxT>(a, B1, lane);
        B2 = load_wave_bounds<T>(a, tile + 2 * stride, wv, q);

        const int jw = wave_jw(Bc);
        const int64_t base = wave_base(Bc);
        const int js = jw < J ? jw : J;
        const T vt0 = Bc.vt0;
        T num[J], den[J];
#pragma unroll
        for (int s = 0; s < J; ++s) {
            num[s] = s < js ? Pc[s] * Rc.v[s] : T(0);
            den[s] = Rc.den[s];
        }
        unsigned long long mask[J];
        auto full = [&](T R, T& N, T& Dn) {
            T n_ = T(0), d_ = T(0);
#pragma unroll
            for (int s = 0; s < J; ++s) {
                mask[s] = 0ull;
                if (s >= js) continue;
                const bool in = num[s] > R * den[s];
                mask[s] = __ballot(in);
                const T w = in ? T(1) : T(0);
                n_ = fmadd(w, num[s], n_);
                d_ = fmadd(w, den[s], d_);
            }
            for (int s = J; s < jw; ++s) {            // slots past the registers
                const int64_t e = base + 64 * s + lane;
                const T nn = rho[i3[e]] * v3[e];
                const T dd = d3[e];
                const T w = nn > R * dd ? T(1) : T(0);
                n_ = fmadd(w, nn, n_);
                d_ = fmadd(w, dd, d_);
            }
            N = group_sum(n_);
            Dn = group_sum(d_);
        };
        auto changed = [&](T R, T Rn) {
            unsigned long long diff = 0ull;
#pragma unroll
            for (int s = 0; s < J; ++s) {
                if (s >= js) break;
                diff |= __ballot(num[s] > Rn * den[s]) ^ mask[s];
            }
            if (jw > J) {
                bool t = false;
                for (int s = J; s < jw; ++s) {
                    const int64_t e = base + 64 * s + lane;
                    const T nn = rho[i3[e]] * v3[e];
                    const T dd = d3[e];
                    t = t || ((nn > Rn * dd) != (nn > R * dd));
                }
                diff |= __ballot(t);
            }
            return diff;
        };
        // Dinkelbach as in process_tiles (same readings, same cycle rule)
        T R = Bc.R0, N, Dn;
        full(R, N, Dn);
        T Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        T pR = R, pN = N, pD = Dn, pRs = Rs;
        unsigned long long diff = 0ull;
        for (int round = 0; round <= kGroup * jw + 1; ++round) {
            diff = changed(R, Rs);
            if (diff == 0ull) break;
            pR = R;
            pN = N;
            pD = Dn;
            pRs = Rs;
            R = Rs;
            full(R, N, Dn);
            Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        }
        if (diff != 0ull) {
            const unsigned long long now = changed(R, Rs);
            const bool cycling = ((now >> (threadIdx.x & 56)) & 0xFFull) != 0ull;
            if (cycling && pRs > Rs) {
                R = pR;
                N = pN;
                Dn = pD;
                Rs = pRs;
            }
        }
        const T Rstar = Rs;
        const T lamD = ratio(Bc.lam, vt0 + Dn) * (T)a.fx_scale;
        double pl = 0.0;   // PSEG: sum r_j q_lj over this lane's sales (q in quanta)
#pragma unroll
        for (int s = 0; s < J; ++s) {
            if (s >= js) break;
            if (num[s] > R * den[s]) {
                const unsigned long long qv = quantum(lamD, Rc.v[s]);
                const int32_t j = Rc.id[s];
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qv;
                add_sale<T>(a, bins, j, qv);
            }
        }
        for (int s = J; s < jw; ++s) {
            const int64_t e = base + 64 * s + lane;
            const T x = v3[e];
            const int32_t j = (int32_t)i3[e];
            if (rho[j] * x > R * d3[e]) {
                const unsigned long long qq = quantum(lamD, x);
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qq;
                add_sale<T>(a, bins, j, qq);
            }
        }
        if constexpr (PSEG) pl = group_sum(pl);
        if ((lane & (kGroup - 1)) == 0 && Bc.live) {
            const int64_t p = (tile * (kSegsPerTile / kGroup) + wv) * kGroup + q;
            zacc.add((double)Bc.lam * (double)Rstar, z_ok((double)Rstar, a.z_rmax), a.z_scale);
            ((T*)a.Rwarm)[p] = Rstar;
            if (a.seg_R) ((T*)a.seg_R)[a.perm[p]] = Rstar;
            if (a.seg_thr) {
                ((T*)a.seg_thr)[p] = R;
                ((T*)a.seg_lamD)[p] = lamD;
            }
            if constexpr (PSEG) a.psum[p] = (a.psum_reset ? 0.0 : a.psum[p]) + pl * a.inv_fx;
        }
        Bc = B1;
        Rc = R1;
        B1 = B2;
    }
}

// ---------------------------------------------------------------------------
// Quad layout: 4-lane groups, 16 rows per wave (wave-tile w = positions
// 16w..16w+15, woff in units of these wave-tiles), entry t of row 16w+q at
// slot t / 4, lane 4q + t % 4.  For short rows this halves the per-row share
// of every per-tile step.  A lane keeps two partial sums, one for the slots of
// even index (the entries an 8-lane group's lane l = t % 8 < 4 would hold) and
// one for the odd slots (lane l + 4), and the quad sum below adds them in the
// order of group_sum, so the results are the 8-lane kernels' bits.
constexpr int kQuad = 4;
constexpr int kQuadRows = 64 / kQuad;                         // rows per wave-tile
constexpr int kQuadTileRows = kSegThreads / 64 * kQuadRows;   // rows per block step

template <typename X>
__device__ __forceinline__ X quad_sum(X lo, X hi)
{
    // lane j of the quad: x_j + x_(7-j) of the 8-lane sum is lo_j + hi_(3-j)
    X x = lo + dpp_move<0x1B>(hi);
    x += dpp_move<kQuadSwap2>(x);
    x += dpp_move<kQuadSwap1>(x);
    return x;
}

// Plain sum over the four lanes of a quad (the same on every lane of it).
__device__ __forceinline__ double quad_total(double x)
{
    x += dpp_move<kQuadSwap2>(x);
    return x + dpp_move<kQuadSwap1>(x);
}

template <typename T>
__device__ __forceinline__ WaveBounds<T> load_wave_bounds_quad(const SegArgs& a, int64_t t, int wv,
                                                              int q)
{
    const int64_t W = (a.L + kQuadRows - 1) / kQuadRows;
    const int64_t w = t * (kSegThreads / 64) + wv;
    const int64_t wc = w < W ? w : 0;
    WaveBounds<T> B;
    B.b0 = a.woff[wc];
    B.b1 = a.woff[wc + 1];
    B.wlive = w < W;
    const int64_t p = w * kQuadRows + q;
    const int64_t pc = p < a.L ? p : 0;
    B.vt0 = ((const T*)a.vt0)[pc];
    B.lam = ((const T*)a.lam)[pc];
    B.R0 = ((const T*)a.Rwarm)[pc];
    B.live = p < a.L;
    return B;
}

template <typename T, int J, typename PR, typename IdxT, bool PSEG = false>
__device__ __forceinline__ void process_tiles_quad(const SegArgs& a, int64_t tile, int64_t tiles,
                                                   int64_t stride, unsigned long long* bins,
                                                   const PR& rho, ZAcc& zacc)
{
    const T* __restrict__ v3 = (const T*)a.v3;
    const T* __restrict__ d3 = (const T*)a.den3;
    const IdxT* __restrict__ i3 = (const IdxT*)a.idx3;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int q = lane / kQuad;
    if (tile >= tiles) return;

    WaveBounds<T> Bc = load_wave_bounds_quad<T>(a, tile, wv, q);
    Raw<T, J> Rc = load_slots<T, J, false, IdxT>(a, Bc, lane);
    WaveBounds<T> B1 = load_wave_bounds_quad<T>(a, tile + stride, wv, q);
    WaveBounds<T> B2;
    T Pc[J];
    for (; tile < tiles; tile += stride) {
        gather<T, J, true, PR>(rho, Rc, Pc, J);
        __builtin_amdgcn_sched_barrier(0);
        const Raw<T, J> R1 = load_slots<T, J, false, IdxT>(a, B1, lane);
        B2 = load_wave_bounds_quad<T>(a, tile + 2 * stride, wv, q);

        const int jw = wave_jw(Bc);
        const int64_t base = wave_base(Bc);
        const int js = jw < J ? jw : J;
        const T vt0 = Bc.vt0;
        T num[J], den[J];
#pragma unroll
        for (int s = 0; s < J; ++s) {
            num[s] = s < js ? Pc[s] * Rc.v[s] : T(0);
            den[s] = Rc.den[s];
        }
        unsigned long long mask[J];
        auto full = [&](T R, T& N, T& Dn) {
            T n0 = T(0), n1 = T(0), d0 = T(0), d1 = T(0);
#pragma unroll
            for (int s = 0; s < J; ++s) {
                mask[s] = 0ull;
                if (s >= js) continue;
                const bool in = num[s] > R * den[s];
                mask[s] = __ballot(in);
                const T w = in ? T(1) : T(0);
                if (s & 1) {
                    n1 = fmadd(w, num[s], n1);
                    d1 = fmadd(w, den[s], d1);
                } else {
                    n0 = fmadd(w, num[s], n0);
                    d0 = fmadd(w, den[s], d0);
                }
            }
            for (int s = J; s < jw; ++s) {            // slots past the registers
                const int64_t e = base + 64 * s + lane;
                const T nn = rho[i3[e]] * v3[e];
                const T dd = d3[e];
                const T w = nn > R * dd ? T(1) : T(0);
                if (s & 1) {
                    n1 = fmadd(w, nn, n1);
                    d1 = fmadd(w, dd, d1);
                } else {
                    n0 = fmadd(w, nn, n0);
                    d0 = fmadd(w, dd, d0);
                }
            }
            N = quad_sum(n0, n1);
            Dn = quad_sum(d0, d1);
        };
        auto changed = [&](T R, T Rn) {
            unsigned long long diff = 0ull;
#pragma unroll
            for (int s = 0; s < J; ++s) {
                if (s >= js) break;
                diff |= __ballot(num[s] > Rn * den[s]) ^ mask[s];
            }
            if (jw > J) {
                bool t = false;
                for (int s = J; s < jw; ++s) {
                    const int64_t e = base + 64 * s + lane;
                    const T nn = rho[i3[e]] * v3[e];
                    const T dd = d3[e];
                    t = t || ((nn > Rn * dd) != (nn > R * dd));
                }
                diff |= __ballot(t);
            }
            return diff;
        };
        // Dinkelbach with the same start, round cap (in entries of the wave's
        // longest row, rounded to 8) and cycle rule as the 8-lane kernels
        T R = Bc.R0, N, Dn;
        full(R, N, Dn);
        T Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        T pR = R, pN = N, pD = Dn, pRs = Rs;
        unsigned long long diff = 0ull;
        const int cap = kGroup * ((kQuad * jw + kGroup - 1) / kGroup) + 1;
        for (int round = 0; round <= cap; ++round) {
            diff = changed(R, Rs);
            if (diff == 0ull) break;
            pR = R;
            pN = N;
            pD = Dn;
            pRs = Rs;
            R = Rs;
            full(R, N, Dn);
            Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        }
        if (diff != 0ull) {
            const unsigned long long now = changed(R, Rs);
            const bool cycling = ((now >> (threadIdx.x & 60)) & 0xFull) != 0ull;
            if (cycling && pRs > Rs) {
                R = pR;
                N = pN;
                Dn = pD;
                Rs = pRs;
            }
        }
        const T Rstar = Rs;
        const T lamD = ratio(Bc.lam, vt0 + Dn) * (T)a.fx_scale;
        double pl = 0.0;   // PSEG: sum r_j q_lj over this lane's sales (q in quanta)
#pragma unroll
        for (int s = 0; s < J; ++s) {
            if (s >= js) break;
            if (num[s] > R * den[s]) {
                const unsigned long long qv = quantum(lamD, Rc.v[s]);
                const int32_t j = Rc.id[s];
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qv;
                add_sale<T>(a, bins, j, qv);
            }
        }
        for (int s = J; s < jw; ++s) {
            const int64_t e = base + 64 * s + lane;
            const T x = v3[e];
            const int32_t j = (int32_t)i3[e];
            if (rho[j] * x > R * d3[e]) {
                const unsigned long long qq = quantum(lamD, x);
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qq;
                add_sale<T>(a, bins, j, qq);
            }
        }
        if constexpr (PSEG) pl = quad_total(pl);
        if ((lane & (kQuad - 1)) == 0 && Bc.live) {
            const int64_t p = (tile * (kSegThreads / 64) + wv) * kQuadRows + q;
            zacc.add((double)Bc.lam * (double)Rstar, z_ok((double)Rstar, a.z_rmax), a.z_scale);
            ((T*)a.Rwarm)[p] = Rstar;
            if (a.seg_R) ((T*)a.seg_R)[a.perm[p]] = Rstar;
            if (a.seg_thr) {
                ((T*)a.seg_thr)[p] = R;
                ((T*)a.seg_lamD)[p] = lamD;
            }
            if constexpr (PSEG) a.psum[p] = (a.psum_reset ? 0.0 : a.psum[p]) + pl * a.inv_fx;
        }
        Bc = B1;
        Rc = R1;
        B1 = B2;
    }
}

// Pair layout: 2-lane groups, 32 rows per wave (entry t of row q at slot
// t / 2, lane 2q + t % 2), for rows of at most 16 entries.  Lane l of a pair
// keeps four partial sums, slots s = 0, 1, 2, 3 (mod 4): the sums of the
// 8-lane lanes l, l + 2, l + 4, l + 6; pair_sum adds them in group_sum's order
// ((x0 + x7) + (x2 + x5)) + ((x1 + x6) + (x3 + x4)), the same on both lanes.
constexpr int kPair = 2;
constexpr int kPairRows = 64 / kPair;
constexpr int kPairTileRows = kSegThreads / 64 * kPairRows;

template <typename X>
__device__ __forceinline__ X pair_sum(const X (&c)[4], int lane)
{
    const bool l0 = (lane & 1) == 0;
    X A[4], B[4];   // the even lane's and the odd lane's partial sums
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const X o = dpp_move<kQuadSwap1>(c[k]);
        A[k] = l0 ? c[k] : o;
        B[k] = l0 ? o : c[k];
    }
    // x(l + 2k) is A[k] for l = 0 and B[k] for l = 1
    const X y0 = A[0] + B[3];   // x0 + x7
    const X y2 = A[1] + B[2];   // x2 + x5
    const X y1 = B[0] + A[3];   // x1 + x6
    const X y3 = B[1] + A[2];   // x3 + x4
    return (y0 + y2) + (y1 + y3);
}

template <typename T>
__device__ __forceinline__ WaveBounds<T> load_wave_bounds_pair(const SegArgs& a, int64_t t, int wv,
                                                              int q)
{
    const int64_t W = (a.L + kPairRows - 1) / kPairRows;
    const int64_t w = t * (kSegThreads / 64) + wv;
    const int64_t wc = w < W ? w : 0;
    WaveBounds<T> B;
    B.b0 = a.woff[wc];
    B.b1 = a.woff[wc + 1];
    B.wlive = w < W;
    const int64_t p = w * kPairRows + q;
    const int64_t pc = p < a.L ? p : 0;
    B.vt0 = ((const T*)a.vt0)[pc];
    B.lam = ((const T*)a.lam)[pc];
    B.R0 = ((const T*)a.Rwarm)[pc];
    B.live = p < a.L;
    return B;
}

template <typename T, int J, typename PR, typename IdxT, bool PSEG = false>
__device__ __forceinline__ void process_tiles_pair(const SegArgs& a, int64_t tile, int64_t tiles,
                                                   int64_t stride, unsigned long long* bins,
                                                   const PR& rho, ZAcc& zacc)
{
    const T* __restrict__ v3 = (const T*)a.v3;
    const T* __restrict__ d3 = (const T*)a.den3;
    const IdxT* __restrict__ i3 = (const IdxT*)a.idx3;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int q = lane / kPair;
    if (tile >= tiles) return;

    WaveBounds<T> Bc = load_wave_bounds_pair<T>(a, tile, wv, q);
    Raw<T, J> Rc = load_slots<T, J, false, IdxT>(a, Bc, lane);
    WaveBounds<T> B1 = load_wave_bounds_pair<T>(a, tile + stride, wv, q);
    WaveBounds<T> B2;
    T Pc[J];
    for (; tile < tiles; tile += stride) {
        gather<T, J, true, PR>(rho, Rc, Pc, J);
        __builtin_amdgcn_sched_barrier(0);
        const Raw<T, J> R1 = load_slots<T, J, false, IdxT>(a, B1, lane);
        B2 = load_wave_bounds_pair<T>(a, tile + 2 * stride, wv, q);

        const int jw = wave_jw(Bc);
        const int64_t base = wave_base(Bc);
        const int js = jw < J ? jw : J;
        const T vt0 = Bc.vt0;
        T num[J], den[J];
#pragma unroll
        for (int s = 0; s < J; ++s) {
            num[s] = s < js ? Pc[s] * Rc.v[s] : T(0);
            den[s] = Rc.den[s];
        }
        unsigned long long mask[J];
        auto full = [&](T R, T& N, T& Dn) {
            T nc[4] = {T(0), T(0), T(0), T(0)}, dc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int s = 0; s < J; ++s) {
                mask[s] = 0ull;
                if (s >= js) continue;
                const bool in = num[s] > R * den[s];
                mask[s] = __ballot(in);
                const T w = in ? T(1) : T(0);
                nc[s & 3] = fmadd(w, num[s], nc[s & 3]);
                dc[s & 3] = fmadd(w, den[s], dc[s & 3]);
            }
            for (int s = J; s < jw; ++s) {            // slots past the registers
                const int64_t e = base + 64 * s + lane;
                const T nn = rho[i3[e]] * v3[e];
                const T dd = d3[e];
                const T w = nn > R * dd ? T(1) : T(0);
                switch (s & 3) {                     // the class of the slot, as a constant index
                case 0: nc[0] = fmadd(w, nn, nc[0]); dc[0] = fmadd(w, dd, dc[0]); break;
                case 1: nc[1] = fmadd(w, nn, nc[1]); dc[1] = fmadd(w, dd, dc[1]); break;
                case 2: nc[2] = fmadd(w, nn, nc[2]); dc[2] = fmadd(w, dd, dc[2]); break;
                default: nc[3] = fmadd(w, nn, nc[3]); dc[3] = fmadd(w, dd, dc[3]); break;
                }
            }
            N = pair_sum(nc, lane);
            Dn = pair_sum(dc, lane);
        };
        auto changed = [&](T R, T Rn) {
            unsigned long long diff = 0ull;
#pragma unroll
            for (int s = 0; s < J; ++s) {
                if (s >= js) break;
                diff |= __ballot(num[s] > Rn * den[s]) ^ mask[s];
            }
            if (jw > J) {
                bool t = false;
                for (int s = J; s < jw; ++s) {
                    const int64_t e = base + 64 * s + lane;
                    const T nn = rho[i3[e]] * v3[e];
                    const T dd = d3[e];
                    t = t || ((nn > Rn * dd) != (nn > R * dd));
                }
                diff |= __ballot(t);
            }
            return diff;
        };
        // Dinkelbach with the same start, round cap (in entries of the wave's
        // longest row, rounded to 8) and cycle rule as the 8-lane kernels
        T R = Bc.R0, N, Dn;
        full(R, N, Dn);
        T Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        T pR = R, pN = N, pD = Dn, pRs = Rs;
        unsigned long long diff = 0ull;
        const int cap = kGroup * ((kPair * jw + kGroup - 1) / kGroup) + 1;
        for (int round = 0; round <= cap; ++round) {
            diff = changed(R, Rs);
            if (diff == 0ull) break;
            pR = R;
            pN = N;
            pD = Dn;
            pRs = Rs;
            R = Rs;
            full(R, N, Dn);
            Rs = N > T(0) ? ratio(N, vt0 + Dn) : T(0);
        }
        if (diff != 0ull) {
            const unsigned long long now = changed(R, Rs);
            const bool cycling = ((now >> (threadIdx.x & 62)) & 0x3ull) != 0ull;
            if (cycling && pRs > Rs) {
                R = pR;
                N = pN;
                Dn = pD;
                Rs = pRs;
            }
        }
        const T Rstar = Rs;
        const T lamD = ratio(Bc.lam, vt0 + Dn) * (T)a.fx_scale;
        double pl = 0.0;   // PSEG: sum r_j q_lj over this lane's sales (q in quanta)
#pragma unroll
        for (int s = 0; s < J; ++s) {
            if (s >= js) break;
            if (num[s] > R * den[s]) {
                const unsigned long long qv = quantum(lamD, Rc.v[s]);
                const int32_t j = Rc.id[s];
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qv;
                add_sale<T>(a, bins, j, qv);
            }
        }
        for (int s = J; s < jw; ++s) {
            const int64_t e = base + 64 * s + lane;
            const T x = v3[e];
            const int32_t j = (int32_t)i3[e];
            if (rho[j] * x > R * d3[e]) {
                const unsigned long long qq = quantum(lamD, x);
                if constexpr (PSEG) pl += (double)((const T*)a.rlib)[j] * (double)(long long)qq;
                add_sale<T>(a, bins, j, qq);
            }
        }
        if constexpr (PSEG) pl = pl + dpp_move<kQuadSwap1>(pl);
        if ((lane & (kPair - 1)) == 0 && Bc.live) {
            const int64_t p = (tile * (kSegThreads / 64) + wv) * kPairRows + q;
            zacc.add((double)Bc.lam * (double)Rstar, z_ok((double)Rstar, a.z_rmax), a.z_scale);
            ((T*)a.Rwarm)[p] = Rstar;
            if (a.seg_R) ((T*)a.seg_R)[a.perm[p]] = Rstar;
            if (a.seg_thr) {
                ((T*)a.seg_thr)[p] = R;
                ((T*)a.seg_lamD)[p] = lamD;
            }
            if constexpr (PSEG) a.psum[p] = (a.psum_reset ? 0.0 : a.psum[p]) + pl * a.inv_fx;
        }
        Bc = B1;
        Rc = R1;
        B1 = B2;
    }
}

}  // namespace seg
}  // namespace cblp

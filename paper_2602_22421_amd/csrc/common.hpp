// Shared declarations of libcblp's kernels and host code (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "cblp.h"

namespace cblp {

// Segment kernel: an 8-lane group (half a DPP row) owns one segment and keeps
// a few products per lane in registers; a block holds kSegThreads / 8
// groups.  Longer rows stream their tail from memory.
constexpr int kGroup = 8;
constexpr int kMaxJ = 8;                   // most register slots of any variant
constexpr int kPad = kGroup * kMaxJ;       // padding entries after the CSR copy
constexpr int kSegThreads = 1024;
constexpr int kSegsPerTile = kSegThreads / kGroup;

// Dual-phase kernels.
constexpr int kFoldLite = 256;             // products per fold block
constexpr int kStepWaves = 8;              // waves of a fused fold-and-step block (64 products)
constexpr int kFoldProducts = 64;          // products per batched fold block
constexpr int kRowThreads = 256;

// Z = sum_l lambda_l R*_l is summed in 64-bit fixed point, so that its sum,
// like the sales sums, does not depend on how segments are grouped into
// blocks or work items.  With duals >= 0 every R*_l is at most the largest
// revenue r_max, and the scale z_scale (a power of two chosen at creation)
// keeps sum_l lambda_l r_max z_scale below 2^60, so no partial sum can
// overflow.  A segment whose R* exceeds r_max (beyond rounding: negative
// duals) or is NaN marks the sum invalid: its partials hold kZPoison and the
// sum reads as NaN.
constexpr long long kZPoison = -0x7fffffffffffffffll - 1;   // INT64_MIN
struct ZAcc {
    long long q = 0;
    bool bad = false;
    // v = lambda R*, ok: R* within [0, r_max (1 + 2^-20)]
    __device__ __forceinline__ void add(double v, bool ok, double zs)
    {
        if (ok)
            q += __double2ll_rn(v * zs);
        else
            bad = true;
    }
};
__device__ __forceinline__ bool z_ok(double R, double rmax) { return R <= rmax; }

// The block's sum of the threads' ZAcc (or kZPoison), returned to every
// thread; sh holds one value per wave.  Integer sums: any order gives the
// same value.
__device__ __forceinline__ long long block_z(const ZAcc& z, long long* sh)
{
    long long q = z.q;
    for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
    const bool bad = __ballot(z.bad) != 0ull;
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = bad ? kZPoison : q;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w)
        t = (t == kZPoison || sh[w] == kZPoison) ? kZPoison : t + sh[w];
    return t;
}

// Z from fixed-point partials [q0, q1) taken by the block's threads in
// strides (every thread gets the value; NaN when a partial is kZPoison).
__device__ __forceinline__ double fold_z(const long long* part, int q0, int q1, double inv_z,
                                         long long* sh)
{
    ZAcc z;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += (int)blockDim.x) {
        const long long v = part[q];
        if (v == kZPoison) z.bad = true; else z.q += v;
    }
    const long long t = block_z(z, sh);
    return t == kZPoison ? __longlong_as_double(0x7ff8000000000000ll) : (double)t * inv_z;
}

// Device-resident solver state (FP64), updated by the finalising block.
struct DevState {
    double dbest, lb, sum_p, scale;
    long long t, t0, cnt, restart;
};

// The segment kernel reads the library's own copy of the instance, with
// segments reordered by consideration-set size (position p holds original
// segment perm[p]) so that neighbouring groups have equal-length rows, and
// products renumbered by falling degree (caller product j is pnew[j]), so
// that the LDS bins and LDS prices of the low ids serve most entries.  The
// price vector rho and the sales accumulators are indexed by these ids.
struct SegArgs {
    int64_t L;
    const int64_t* ptr;            // [L+1] row pointers of the sorted layout
    const int32_t* idx;            // [nnz] product ids
    const void* v;                 // [nnz] nominal attraction
    const void* den;               // [nnz] v - w
    const void* vt0;               // [L] v0 + sum w
    const void* lam;               // [L] arrival rates
    void* Rwarm;                   // [L] last R* per position: Dinkelbach start
    const int32_t* perm;           // [L] position -> original segment
    const void* rho;               // [n] reduced revenues
    int64_t n;                     // products (length of rho)
    int H;                         // products [0, H) are summed in LDS bins:
    int H64;                       // [0, H64) in 64-bit ones, [H64, H) in 32-bit
                                   // ones after them (FP32 quanta only)
    int hp;                        // split-price kernel: prices [0, hp) held in LDS
    unsigned long long* S_fx;      // [n] fixed-point sales of products >= H
    unsigned long long* brow;      // nullable: each block's bins as one row of
    int64_t row_words;             // row_words 64-bit words (else atomics into S_fx)
    double fx_scale;               // 2^bits; one segment's sale * 2^bits < 2^31 for FP32
    long long* zpart;              // [gridDim.x] fixed-point partials of sum lambda R* (or kZPoison)
    double z_scale;                // their scale
    double z_rmax;                 // r_max (1 + 2^-20): the largest R* of duals >= 0
    void* seg_R;                   // [L] nullable, original segment order
    void* seg_thr;                 // [L] nullable, by position: the threshold R of S* =
                                   // {rho v > R den} (evaluation, per-entry sales)
    void* seg_lamD;                // [L] with seg_thr: (lambda / D) 2^bits of the position
    // per-segment certified bound: revenue of each position's best response
    // added to psum[p] (overwritten instead when psum_reset), in the kernels
    // instantiated for it; rlib [n] holds the revenues by library product id
    double* psum;
    const void* rlib;
    double inv_fx;                 // 2^-bits
    int psum_reset;
    // slot-major copy (slot-major kernels): wave-tile w (positions 8w..8w+7)
    // holds (woff[w+1] - woff[w]) / 64 slots of 64 entries from woff[w]
    const int64_t* woff;           // [ceil(L/8) + 2], the last entry repeats the total
    const void* idx3;              // int32 ids, or uint16 for the 16-bit-id kernels
    const void* v3;
    const void* den3;
};

struct PhaseArgs {
    int64_t n, m;
    int mode;                      // 0: iterate, 1: evaluate at fixed eta, 2: minibatch
                                   // iterate (dual step only, no certificate)
    int keep_sales;                // the sales totals S_fx persist (minibatch running sums)
    int rule, check_every;
    double gamma, mu, tau_s;
    double tau_mult;               // CONST: the step multiplier of this iteration (decay)
    const void* tau_vec;           // [m] nullable
    const long long* zpart;        // fixed-point partials of Z (scale 1 / inv_z), kZPoison: invalid
    double inv_z;
    int nz;
    unsigned long long* S_fx;
    double inv_fx;
    const void* r;
    const void* c;
    const int64_t* a_ptr;          // CSC of A by product; NULL: identity
    const int32_t* a_idx;
    const void* a_val;
    const int64_t* at_ptr;         // CSR of A by resource
    const int32_t* at_prod;
    const double* at_val;
    void* eta;
    void* rho;
    double* S_d;
    double* u_d;
    double* sum_u;
    double* bpart;                 // [fold blocks][8]
    double* bpart2;                // [row blocks][8]
    int fold_blocks;
    const int32_t* pnew;           // [n] library product id of caller product j; NULL: j
    const int32_t* pinv;           // [n] caller product of library id q; NULL: q
    // the segment blocks' rows of sales bins still to add (nrows 0: none):
    // row r at brow + r * row_words, 64-bit bins of library ids [0, rows_H64),
    // then 32-bit ones of [rows_H64, rows_H)
    const unsigned long long* brow;
    int64_t row_words;
    int nrows, rows_H, rows_H64;
    unsigned* arrive;              // blocks of the fused fold-and-step kernel done (0 between launches)
    DevState* st;                  // [2]: read st[par], write st[par ^ 1]
    int par;
    double* row;                   // trace row of this iteration
    // per-segment bound (check iterations only; pseg_part NULL otherwise):
    // theta_prod [n] by library id, the position-ordered copy (L, ptr2,
    // idx2 with library ids) and psum [L]; one partial per k_pseg block
    double* theta_prod;
    int64_t L;
    const int64_t* ptr2;
    const int32_t* idx2;
    const double* psum;
    double* pseg_part;
    int pseg_blocks;
};

// Launchers (one per kernel family), defined next to their kernels.
template <typename T>
hipError_t launch_validate(int64_t L, int64_t n, int64_t m, int64_t nnz, int64_t nnzA,
                           const int64_t* seg_ptr, const int32_t* idx, const void* v,
                           const void* w, const void* v0, const void* lam, const void* r,
                           const void* c, const int64_t* a_ptr, const int32_t* a_idx,
                           const void* a_val, unsigned* flags, hipStream_t s);
template <typename T>
hipError_t launch_prepare(int64_t L, const void* lam, double* lam_part, int blocks,
                          hipStream_t s);   // lam_part[2 * block] = sum, [2 * block + 1] = max
template <typename T>
hipError_t launch_relayout(int64_t L, const int64_t* seg_ptr, const int32_t* idx,
                           const void* v, const void* w, const void* v0, const void* lam,
                           const int32_t* perm, const int32_t* pnew, const int64_t* ptr,
                           int32_t* idx2, void* v2, void* den2, void* vt0, void* lam2, void* Rwarm,
                           void* v0c, hipStream_t s);
// deg[j] = number of entries with product j (zeroes deg first)
hipError_t launch_degree(int64_t nnz, const int32_t* idx, int64_t n, unsigned long long* deg,
                         hipStream_t s);
template <typename T>
// G: lanes per row of the layout (8, 4: quad, 2: pair)
hipError_t launch_relayout_slots(int64_t L, const int64_t* ptr, const int32_t* idx2,
                                 const void* v2, const void* den2, const int64_t* woff,
                                 int64_t entries, void* idx3, bool idx16, int G, void* v3,
                                 void* den3, hipStream_t s);
template <typename T>
hipError_t launch_prices(int64_t n, const void* r, const void* eta, const int64_t* a_ptr,
                         const int32_t* a_idx, const void* a_val, const int32_t* pnew, void* rho,
                         hipStream_t s);
// Segment kernels (segment.hip).  Every one reads the slot-major copy (see
// SegArgs::woff) and gives the same bits as the others.
//   kSegMixed3         FP32, three parts (2-, 4- and 8-lane groups), all n
//                      prices in LDS, 16-bit product ids (n <= 65536)
//   kSegMixed3Split16  the same with only the prices of products [0, hp) in
//                      LDS, the rest read from global memory
//   kSegMixed3Split32  the same with 32-bit product ids
//   kSegSlots16        FP64, 8-lane groups, 4 register slots, prices from
//                      global memory, 16-bit ids
//   kSegSlots32        the same with 32-bit ids
enum {
    kSegMixed3 = 0,
    kSegMixed3Split16 = 1,
    kSegMixed3Split32 = 2,
    kSegSlots16 = 3,
    kSegSlots32 = 4,
    kSegVariants = 5
};
constexpr int kQuadMaxRow = 32;        // rows held in registers by the 4-lane groups
constexpr int kPairMaxRow = 16;        // rows held in registers by the 2-lane groups
constexpr int kSplitPrices = 16384;    // head prices held in LDS by the split kernels
inline bool seg_mixed3(int variant) { return variant <= kSegMixed3Split32; }
inline bool seg_split(int variant)
{
    return variant == kSegMixed3Split16 || variant == kSegMixed3Split32;
}
inline bool seg_idx16(int variant) { return variant != kSegMixed3Split32 && variant != kSegSlots32; }
inline bool seg_lds_prices(int variant) { return seg_mixed3(variant); }
// bytes of a block's LDS bins: H64 64-bit ones, then H - H64 32-bit ones,
// rounded up to 8
__host__ __device__ inline size_t seg_bin_bytes(int H, int H64)
{
    return ((size_t)H64 * 8 + (size_t)(H - H64) * 4 + 7) & ~(size_t)7;
}
// dynamic LDS bytes of a segment block: the bins, then the prices held in
// LDS (n of them, or hp for the split kernels)
inline size_t seg_lds_bytes(int H, int H64, int64_t n, int hp, size_t esz, int variant)
{
    const size_t np = seg_split(variant) ? (size_t)hp : seg_lds_prices(variant) ? (size_t)n : 0;
    return seg_bin_bytes(H, H64) + np * esz;
}
// a2, a4, a8: views of the pair, quad and 8-lane parts of the slot-major
// copy (the FP64 kernels take a8 only, viewing the whole instance)
// pseg: the kernels that also add each segment's revenue to a2.psum etc.
template <typename T>
hipError_t launch_segments(const SegArgs& a2, const SegArgs& a4, const SegArgs& a8, int grid,
                           int variant, bool pseg, hipStream_t s);
// s_out [nnz] (caller's CSR order) from the thresholds and (lambda / D) 2^bits
// that a segment pass stored by position (thr, lamD)
template <typename T>
hipError_t launch_entry_sales(int64_t L, const int32_t* perm, const int64_t* seg_ptr,
                              const int32_t* idx, const void* v, const void* w,
                              const int32_t* pnew, const void* rho, const void* thr,
                              const void* lamD, double inv_fx, double* s_out, hipStream_t s);
template <typename T>
int segment_blocks_per_cu(int H, int H64, int64_t n, int hp, int variant);   // resident blocks per CU
// FP32 copies: need = 1 + the largest product id < Hc whose sales within one
// of the G segment blocks may reach 2^32 quanta (0 if none); Ub is zeroed
// [Hc x G] scratch, need a zeroed int
hipError_t launch_bin_bound(int64_t L, int64_t P2, int64_t P4, int G, const int64_t* ptr2,
                            const int32_t* idx2, const void* v2, const void* den2,
                            const void* vt0, const void* lam, double fx_scale, int Hc,
                            unsigned long long* Ub, int* need, hipStream_t s);
// The sum, as a 64-bit integer, of bin q in rows first, first + stride, ...
// below nrows of a segment pass's block rows (0 for q >= H): the loads of up
// to 16 rows are in flight together.
__device__ __forceinline__ unsigned long long row_bins_sum(const unsigned long long* __restrict__ rows,
                                                           int64_t row_words, int nrows, int H,
                                                           int H64, int64_t q, int first, int stride)
{
    constexpr int kU = 16;
    unsigned long long acc = 0ull;
    if (q >= H) return acc;
    if (q < H64) {
        const unsigned long long* p = rows + q;
        for (int r0 = first; r0 < nrows; r0 += stride * kU) {
            unsigned long long x[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int r = r0 + u * stride;
                x[u] = r < nrows ? p[(int64_t)r * row_words] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) acc += x[u];
        }
    } else {
        const unsigned* p = (const unsigned*)(rows + H64) + (q - H64);
        for (int r0 = first; r0 < nrows; r0 += stride * kU) {
            unsigned x[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int r = r0 + u * stride;
                x[u] = r < nrows ? p[(int64_t)r * row_words * 2] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) acc += x[u];
        }
    }
    return acc;
}
template <typename T>
hipError_t launch_phase(const PhaseArgs& a, bool identity, hipStream_t s);
constexpr int kPsegBlocks = 256;   // blocks of the per-segment bound pass

// Record a failure for cblp_last_error() on this thread; returns code.
int set_error(int code, const std::string& msg);

enum : unsigned {
    V_IDX = 1u << 0, V_V = 1u << 1, V_W = 1u << 2, V_V0 = 1u << 3, V_LAM = 1u << 4,
    V_SEGPTR = 1u << 5, V_R = 1u << 6, V_C = 1u << 7, V_AIDX = 1u << 8, V_AVAL = 1u << 9,
    V_APTR = 1u << 10, V_NBITS = 11
};

}  // namespace cblp

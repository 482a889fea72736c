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
constexpr int kFoldProducts = 64;          // products per fold block
constexpr int kFoldChunks = 16;            // partial rows split 16 ways
constexpr int kFoldThreads = kFoldProducts * kFoldChunks;
constexpr int kRowThreads = 256;

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
    int H;                         // products [0, H) are summed in LDS bins
    int hp;                        // split-price kernel: prices [0, hp) held in LDS
    unsigned long long* part_S;    // [gridDim.x][H] per-block bin totals
    unsigned long long* S_fx;      // [n] fixed-point sales of products >= H
    double fx_scale;               // 2^bits; one segment's sale * 2^bits < 2^31 for FP32
    double* zpart;                 // [gridDim.x] FP64 partials of sum lambda R*
    void* seg_R;                   // [L] nullable, original segment order
    const int64_t* blk;            // [grid][3] (slots J, first tile, end tile) of each
                                   // block for the size-class kernels, else unused
    // slot-major copy (slot-major kernels): wave-tile w (positions 8w..8w+7)
    // holds (woff[w+1] - woff[w]) / 64 slots of 64 entries from woff[w]
    const int64_t* woff;           // [ceil(L/8) + 2], the last entry repeats the total
    const void* idx3;              // int32 ids, or uint16 for the 16-bit-id kernels
    const void* v3;
    const void* den3;
};

struct PhaseArgs {
    int64_t n, m;
    int mode;                      // 0: iterate, 1: evaluate at fixed eta
    int rule, check_every;
    double gamma, mu, tau_s;
    const void* tau_vec;           // [m] nullable
    const double* zpart;
    int nz;
    const unsigned long long* part_S;
    int nseg;
    int H;
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
    unsigned* arrive;              // blocks of the fused fold-and-step kernel done (0 between launches)
    DevState* st;                  // [2]: read st[par], write st[par ^ 1]
    int par;
    double* row;                   // trace row of this iteration
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
// Segment-kernel variants 0-9 gather prices from global memory; variants
// kSegLdsPrices and up first copy the n prices into LDS after the H bins.
// Variants kSegClassLds (prices in LDS) and kSegClassGlobal take the slot
// count of each block from a table: blocks own runs of tiles of one size class.
// Variant kSegSplit holds the prices of products [0, hp) in LDS.  Variants
// kSegSlots and up read the slot-major copy (see SegArgs::woff); of these,
// kSegSlotsSplit and kSegSlotsSplit + 1 hold the prices as kSegSplit does.
constexpr int kSegVariants = 41;
constexpr int kSegSlots = 20;
constexpr int kSegSlotsSplit = 26;
constexpr int kSegSlotsJ4 = 28;        // 4 register slots, prices in LDS
// as kSegSlots + 1, kSegSlotsJ4 and kSegSlots + 3 with 16-bit product ids in
// the slot-major copy (n <= 65536): 10 bytes per FP32 entry instead of 12,
// 18 per FP64 entry instead of 20
constexpr int kSegSlots16 = 29;
// quad layout (4-lane groups, 16 rows per wave; rows of at most 32 entries
// in registers): 32 16-bit ids and LDS prices, 33 32-bit ids and split
// prices, 34 32-bit ids and LDS prices
constexpr int kSegQuad = 32;
inline bool seg_quad(int variant) { return variant >= kSegQuad && variant <= kSegQuad + 2; }
// mixed: rows of at most 32 entries in the quad layout, longer rows in the
// 8-lane one, prices in LDS (35: 16-bit ids, 36: 32-bit ids)
constexpr int kSegMixed = 35;
constexpr int kQuadMaxRow = 32;        // rows held in registers by the quad kernels
inline bool seg_mixed(int variant) { return variant == kSegMixed || variant == kSegMixed + 1; }
// three-part mixed: rows of at most 16 entries in the pair layout (2-lane
// groups), then quad, then 8-lane (37: 16-bit ids, 38: 32-bit ids; 39, 40:
// the same with split prices, 32- and 16-bit ids)
constexpr int kSegMixed3 = 37;
constexpr int kPairMaxRow = 16;
inline bool seg_mixed3(int variant) { return variant >= kSegMixed3 && variant <= kSegMixed3 + 3; }
inline bool seg_idx16(int variant)
{
    return (variant >= kSegSlots16 && variant <= kSegSlots16 + 2) || variant == kSegQuad ||
           variant == kSegMixed || variant == kSegMixed3 || variant == kSegMixed3 + 3;
}
inline bool seg_slot_major(int variant) { return variant >= kSegSlots; }
constexpr int kSegLdsPrices = 10;
constexpr int kSegClassLds = 17, kSegClassGlobal = 18, kSegSplit = 19;
constexpr int kSplitPrices = 8192;     // head prices of the split kernel
inline bool seg_split(int variant)
{
    return variant == kSegSplit || variant == kSegSlotsSplit || variant == kSegSlotsSplit + 1 ||
           variant == kSegQuad + 1 || variant == kSegMixed3 + 2 || variant == kSegMixed3 + 3;
}
inline bool seg_class(int variant) { return variant == kSegClassLds || variant == kSegClassGlobal; }
// most register slots of the size-class kernels per element size
inline int seg_class_max_slots(size_t esz) { return esz == 4 ? 7 : 4; }
inline bool seg_lds_prices(int variant)
{
    return variant >= kSegLdsPrices && variant != kSegClassGlobal && variant != kSegSlots + 3 &&
           variant != kSegSlots + 5 && variant != kSegSlots16 + 2;
}
// dynamic LDS bytes of a segment block: H bins, then the prices if in LDS
inline size_t seg_lds_bytes(int H, int64_t n, size_t esz, int variant)
{
    return (size_t)H * 8 + (seg_lds_prices(variant) ? (size_t)n * esz : 0);
}
template <typename T>
hipError_t launch_segments(const SegArgs& a, int grid, int variant, hipStream_t s);
// mixed variants: a = the quad part (positions [0, P)), b = the rest
template <typename T>
hipError_t launch_segments_mixed(const SegArgs& a, const SegArgs& b, int grid, int variant,
                                 hipStream_t s);
// three-part mixed variants: pair, quad and 8-lane parts
template <typename T>
hipError_t launch_segments_mixed3(const SegArgs& a2, const SegArgs& a4, const SegArgs& a8, int grid,
                                  int variant, hipStream_t s);
template <typename T>
int segment_blocks_per_cu(int H, int64_t n, int variant);   // resident blocks per CU
template <typename T>
hipError_t launch_phase(const PhaseArgs& a, bool identity, hipStream_t s);

// Record a failure for cblp_last_error() on this thread; returns code.
int set_error(int code, const std::string& msg);

enum : unsigned {
    V_IDX = 1u << 0, V_V = 1u << 1, V_W = 1u << 2, V_V0 = 1u << 3, V_LAM = 1u << 4,
    V_SEGPTR = 1u << 5, V_R = 1u << 6, V_C = 1u << 7, V_AIDX = 1u << 8, V_AVAL = 1u << 9,
    V_APTR = 1u << 10, V_NBITS = 11
};

}  // namespace cblp

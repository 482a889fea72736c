// The solver handle behind cblp_t (host struct; device buffers it owns).
#pragma once

#include <cstdint>
#include <utility>
#include <vector>

#include "common.hpp"

namespace cblp {
// Part boundaries of the mixed slot-major copies are multiples of this many
// positions (a tile of the pair layout), so that every part, and every batch
// work item, starts on a tile of every layout.
constexpr int64_t kPartAlign = 512;
}  // namespace cblp

struct cblp_instance {
    int device = 0;
    int dtype = CBLP_F32;
    size_t esz = 4;
    int64_t L = 0, n = 0, m = 0, nnz = 0, nnzA = 0;
    const int64_t* seg_ptr = nullptr;
    const int32_t* idx = nullptr;
    const void *v = nullptr, *w = nullptr, *v0 = nullptr, *lam = nullptr;
    const void *r = nullptr, *c = nullptr;
    const int64_t* a_ptr = nullptr;
    const int32_t* a_idx = nullptr;
    const void* a_val = nullptr;
    // owned: the size-sorted copy of the segments (position p = segment perm[p])
    int64_t* ptr2 = nullptr;
    int32_t* idx2 = nullptr;
    void* v2 = nullptr;
    void* den2 = nullptr;
    void* vt0 = nullptr;
    void* lam2 = nullptr;
    void* Rwarm = nullptr;
    void* v0c = nullptr;            // v0 per position (features only)
    int32_t* perm = nullptr;
    int64_t* seg_blk = nullptr;     // [seg_grid][3] size-class block table (class variants)
    int64_t* woff = nullptr;        // slot-major copy (slot-major variants): wave-tile offsets
    void* idx3 = nullptr;           // int32, or uint16 when idx16
    int64_t pair_end = 0;           // three-part mixed: positions [0, pair_end) in the pair layout
    int64_t quad_end = 0;           // mixed: positions [pair_end, quad_end) in the quad layout
    int64_t woff_q = 0;             // three-part mixed: index in woff of the quad part's offsets
    int64_t woff_b = 0;             // mixed: index in woff of the 8-lane part's offsets
    bool idx16 = false;
    void* v3 = nullptr;
    void* den3 = nullptr;
    // owned workspace
    void* rho = nullptr;
    unsigned long long* S_fx = nullptr;
    int32_t* pnew = nullptr;        // [n] library id of caller product j (null: ids kept)
    unsigned long long* part_S = nullptr;
    double* S_d = nullptr;
    double* u_d = nullptr;
    double* sum_u = nullptr;
    double* zpart = nullptr;
    double* bpart = nullptr;
    double* bpart2 = nullptr;
    unsigned* arrive = nullptr;     // arrival counter of the fused fold-and-step kernel
    cblp::DevState* st = nullptr;   // [2], double-buffered
    double* trace = nullptr;
    int64_t trace_rows = 0;
    int64_t* at_ptr = nullptr;
    int32_t* at_prod = nullptr;
    double* at_val = nullptr;
    double* pinned = nullptr;
    int seg_grid = 1;
    int seg_variant = 0;
    int H = 0;
    int hp = 0;                     // split-price kernel: prices held in LDS
    bool flush_atomic = true;       // segment blocks add their bins to S_fx by atomics
                                    // (false: per-block partial rows folded by k_fold)
    int fold_blocks = 1;
    double fx_scale = 1.0;
    int64_t t = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;
};


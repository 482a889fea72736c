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
    int64_t* woff = nullptr;        // slot-major copy: wave-tile offsets
    void* idx3 = nullptr;           // int32, or uint16 when idx16
    int64_t pair_end = 0;           // three-part mixed: positions [0, pair_end) in the pair layout
    int64_t quad_end = 0;           // three-part mixed: positions [pair_end, quad_end) in the quad layout
    int64_t woff_q = 0;             // three-part mixed: index in woff of the quad part's offsets
    int64_t woff_b = 0;             // three-part mixed: index in woff of the 8-lane part's offsets
    bool idx16 = false;
    int64_t slot_entries = 0;       // places of the slot-major copy (rows padded to their wave-tile)
    void* v3 = nullptr;
    void* den3 = nullptr;
    // owned workspace
    void* rho = nullptr;
    unsigned long long* S_fx = nullptr;
    int32_t* pnew = nullptr;        // [n] library id of caller product j (null: ids kept)
    int32_t* pinv = nullptr;        // [n] caller product of library id q (null with pnew)
    double* S_d = nullptr;
    double* u_d = nullptr;
    double* sum_u = nullptr;
    long long* zpart = nullptr;     // fixed-point Z partials, one per segment block
    unsigned long long* brow = nullptr;   // [seg_grid x row_words] the blocks' bins
    int64_t row_words = 0;
    double z_scale = 1.0;           // their scale (a power of two)
    double z_rmax = 0.0;            // largest revenue times (1 + 2^-20)
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
    // per-segment bound (allocated on first use): revenues by library id,
    // running revenue sums by position, theta by library id, k_pseg partials
    void* rlib = nullptr;
    double* psum = nullptr;
    double* theta_prod = nullptr;
    double* pseg_part = nullptr;
    int64_t t0h = 0;                // start of the current averaging window (host copy)
    bool psum_reset_next = true;    // the next accumulating pass starts a new window
    bool pseg_window_ok = true;     // every pass of the current window accumulated psum
    // per-entry sales (allocated on first use): threshold and (lambda / D) 2^bits
    // by position
    void* eval_thr = nullptr;
    void* eval_lamD = nullptr;
    // stochastic minibatch state (allocated on first use): per-entry sales in
    // quanta, running product totals, segment positions, sampling stamps
    void* mb_ent = nullptr;           // [nnz] entry records with the kept sales
    unsigned long long* mb_S = nullptr;
    void* mb_rec = nullptr;           // [L] 32-byte per-segment records
    int* mb_stamp = nullptr;
    unsigned* mb_err = nullptr;
    int mb_it = 0;                  // iterations run, for the stamps
    bool mb_clear = true;           // the sales must be cleared before the next use
    int seg_grid = 1;
    int seg_variant = 0;
    int H = 0;                      // products with LDS bins in the segment kernel,
    int H64 = 0;                    // of which 64-bit ones (the rest 32-bit)
    int Hb = 0;                     // 64-bit LDS bins of the batched kernels
    int64_t bin_bytes = 0;          // LDS bytes a segment block has for its bins
    bool bins_stale = true;         // the values changed: choose H, H64 again
    bool fold_pending = false;      // a segment pass left rows for the dual phase to fold
    int hp = 0;                     // split-price kernel: prices held in LDS
    int fold_blocks = 1;
    double fx_scale = 1.0;
    int64_t t = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;
};


namespace cblp {
// Re-read the caller's v, w (and check c) into the handle's copies, on the
// structure of creation; invalid values set validation bits in *flags.
template <typename T>
hipError_t launch_refresh(const cblp_instance* h, unsigned* flags, hipStream_t s);
// Launch the refresh of h on s (flags: a device word the caller clears and
// reads); also marks the handle's kept per-entry minibatch sales stale.
int refresh_launch(cblp_instance* h, unsigned* flags, hipStream_t s);
// Reset the handle's solver state (as spfom_reset).
int reset_handle_state(cblp_instance* h, hipStream_t s);
// The text of validation bits, for error messages.
std::string validation_message(unsigned flags);
// The handles a batch was built over, in order.
const std::vector<cblp_instance*>& batch_handles(cblp_batch_t b);
}  // namespace cblp

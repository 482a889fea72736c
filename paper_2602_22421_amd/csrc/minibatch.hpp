// Stochastic minibatch segment pass (minibatch.hip): its arguments and
// launchers.
#pragma once

#include "common.hpp"

namespace cblp {

// Re-solves the segments batch[0, B) (caller ids) of iteration `it` and adds
// each entry's change of sale to the running product totals S_run.
struct MbArgs {
    int64_t L, B;
    int it;                        // iteration number (duplicate detection)
    const int32_t* batch;          // [B] caller segment ids
    const void* rec;               // [L] per caller segment: row, position, v_t0, lambda
    void* ent;                     // [nnz] per entry (row-major library order): product
                                   // id, v, denominator weight, kept sale in quanta
    void* Rwarm;
    const void* rho;
    double fx_scale;
    int H;                         // products [0, H) accumulate in LDS first
    unsigned long long* S_run;     // [n] running totals (library ids)
    int* stamp;                    // [L] last iteration that sampled each segment
    unsigned* err;                 // bit 0: id out of range, bit 1: id listed twice
};
template <typename T>
hipError_t launch_minibatch(const MbArgs& a, hipStream_t s);
// LDS bins of the minibatch kernel for n products
template <typename T>
int minibatch_bins(int64_t n);
hipError_t launch_minibatch_init(int64_t L, int* stamp, hipStream_t s);
// bytes of a segment's and of an entry's record
constexpr size_t kMbRecBytes = 32;
template <typename T>
constexpr size_t mb_ent_bytes() { return sizeof(T) == 4 ? 16 : 32; }
// the records of the minibatch kernel: one per segment, one per entry with
// its kept sale set to 0 (y^0 = 0); rebuilt whenever the minibatch state
// restarts, since the values may have changed
template <typename T>
hipError_t launch_minibatch_records(int64_t L, const int32_t* perm, const int64_t* ptr2,
                                    const void* vt0, const void* lam, void* rec,
                                    int64_t nnz, const int32_t* idx2, const void* v2,
                                    const void* den2, void* ent, hipStream_t s);

}  // namespace cblp

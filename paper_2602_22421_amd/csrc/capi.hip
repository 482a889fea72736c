// libcblp host side: the C ABI of include/cblp.h.
//
// One SPFOM iteration (Algorithm 3 with every segment sampled, dual step
// eq. 16) is a short fixed sequence of launches on the caller's stream:
//   k_segments                 per-segment best responses and sales scatter
//   k_fold [k_rows] k_update   sales totals, FP64 reductions, dual step
//   [k_prices_after]           rho = r - A^T eta for a general A
// Nothing is read back per iteration; spfom_solve copies one 80-byte trace
// row to pinned host memory every check_every iterations.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"
#include "handle.hpp"
#include "minibatch.hpp"

using namespace cblp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

}  // namespace

int cblp::set_error(int code, const std::string& msg) { return fail(code, msg); }

namespace {

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(CBLP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

const char* kValidationText[V_NBITS] = {
    "product index outside [0, n)", "attraction v not finite and > 0",
    "shadow attraction w outside [0, v)", "no-purchase attraction v0 not finite and > 0",
    "arrival rate lambda not finite and >= 0", "seg_ptr not non-decreasing from 0 to nnz",
    "revenue r not finite", "capacity c not finite and >= 0",
    "resource index outside [0, m)", "resource weight a not finite and >= 0",
    "a_ptr not non-decreasing from 0 to nnzA"};

// LDS bins per segment block: at most this many, and at most what one block
// may allocate besides its static shared memory.
constexpr int kMaxBins = 16384;

}  // namespace


namespace {

template <typename P>
int dalloc(P** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc((void**)p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CBLP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return CBLP_OK;
}

void release(cblp_instance* h)
{
    if (!h) return;
    void* ptrs[] = {h->ptr2, h->idx2, h->v2, h->den2, h->vt0, h->lam2, h->Rwarm, h->v0c, h->perm,
                    h->pnew, h->pinv,
                    h->woff, h->idx3, h->v3, h->den3,
                    h->rho, h->S_fx, h->S_d, h->u_d, h->sum_u, h->zpart, h->brow,
                    h->bpart, h->bpart2, h->st, h->arrive, h->trace, h->at_ptr,
                    h->at_prod, h->at_val, h->rlib, h->psum, h->theta_prod, h->pseg_part,
                    h->eval_thr, h->eval_lamD, h->mb_ent, h->mb_S, h->mb_rec, h->mb_stamp,
                    h->mb_err};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

int timed_begin(cblp_instance* h, int kernel, hipStream_t s, size_t* slot)
{
    *slot = SIZE_MAX;
    if (!h->timing) return CBLP_OK;
    while (h->ev_pool.size() < h->ev_used + 2) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->ev_pool.push_back(e);
    }
    *slot = h->ev_used;
    h->ev_used += 2;
    h->ev_marks.emplace_back(kernel, *slot);
    HIP_TRY(hipEventRecord(h->ev_pool[*slot], s));
    return CBLP_OK;
}

int timed_end(cblp_instance* h, size_t slot, hipStream_t s)
{
    if (slot == SIZE_MAX) return CBLP_OK;
    HIP_TRY(hipEventRecord(h->ev_pool[slot + 1], s));
    return CBLP_OK;
}

int ensure_trace(cblp_instance* h, int64_t rows)
{
    if (rows <= h->trace_rows) return CBLP_OK;
    if (h->trace) (void)hipFree(h->trace);
    h->trace = nullptr;
    h->trace_rows = 0;
    int rc = dalloc(&h->trace, (size_t)rows * SPFOM_NTRACE * sizeof(double));
    if (rc) return rc;
    h->trace_rows = rows;
    return CBLP_OK;
}

int check_params(const spfom_params* p)
{
    if (!p) return fail(CBLP_EINVAL, "params is NULL");
    if (p->rule != SPFOM_STEP_CONST && p->rule != SPFOM_STEP_POLYAK)
        return fail(CBLP_EINVAL, "unknown step rule");
    if (p->check_every < 1) return fail(CBLP_EINVAL, "check_every must be >= 1");
    if (!p->tau_vec && !(p->tau > 0.0 && std::isfinite(p->tau)))
        return fail(CBLP_EINVAL, "tau must be finite and > 0");
    if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) return fail(CBLP_EINVAL, "mu must be >= 0");
    if (p->rule == SPFOM_STEP_POLYAK && !(p->gamma > 0.0 && p->gamma <= 2.0))
        return fail(CBLP_EINVAL, "gamma must be in (0, 2]");
    if (p->bound != SPFOM_BOUND_GLOBAL && p->bound != SPFOM_BOUND_SEGMENT)
        return fail(CBLP_EINVAL, "unknown bound");
    if (!(p->tau_decay >= 0.0 && p->tau_decay <= 1.0))
        return fail(CBLP_EINVAL, "tau_decay must be in [0, 1]");
    if (p->tau_decay > 0.0 && p->tau_decay < 1.0 && p->decay_every < 1)
        return fail(CBLP_EINVAL, "decay_every must be >= 1");
    return CBLP_OK;
}

// The constant step's multiplier in iteration t1 (1-based, since the last
// reset): tau_decay^k with k = (t1 - 1) / decay_every, by repeated FP64
// multiplication (the oracle forms it the same way).
double tau_multiplier(const spfom_params* p, int64_t t1)
{
    if (!p || p->rule != SPFOM_STEP_CONST || !(p->tau_decay > 0.0 && p->tau_decay < 1.0))
        return 1.0;
    const int64_t k = (t1 - 1) / p->decay_every;
    double m = 1.0;
    for (int64_t q = 0; q < k; ++q) m *= p->tau_decay;
    return m;
}

// Buffers of the per-segment bound, made on first use: revenues by library
// product id (r - A^T 0 through the price kernel), the running revenue sums
// by position, theta by library id and the k_pseg partials.
template <typename T>
int ensure_pseg(cblp_instance* h, hipStream_t s)
{
    if (h->psum) return CBLP_OK;
    int rc;
    void* zeros = nullptr;
    if ((rc = dalloc(&zeros, (size_t)h->m * h->esz))) return rc;
    if ((rc = dalloc(&h->rlib, (size_t)h->n * h->esz)) ||
        (rc = dalloc(&h->theta_prod, (size_t)h->n * 8)) ||
        (rc = dalloc(&h->pseg_part, (size_t)kPsegBlocks * 8)) ||
        (rc = dalloc(&h->psum, (size_t)std::max<int64_t>(h->L, 1) * 8))) {
        (void)hipFree(zeros);
        return rc;
    }
    hipError_t e = hipMemsetAsync(zeros, 0, (size_t)h->m * h->esz, s);
    if (e == hipSuccess)
        e = launch_prices<T>(h->n, h->r, zeros, h->a_ptr, h->a_idx, h->a_val, h->pnew, h->rlib, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(zeros);
    if (e != hipSuccess) return fail(CBLP_EHIP, std::string("revenue copy: ") + hipGetErrorString(e));
    return CBLP_OK;
}

// pseg: add each segment's revenue to h->psum (per-segment bound);
// eval_out: store each position's threshold and (lambda / D) 2^bits
// The LDS bins of the segment kernel (FP32 handles with more products than
// 64-bit bins): the products whose sales within every segment block are
// bounded below 2^32 quanta may take 32-bit bins, so the block holds 64-bit
// bins for products [0, need) (the most popular ids), 32-bit ones after them
// up to what its LDS holds; the 64-bit layout stays when that covers more
// products.  Run once the values are known, again after a refresh.
template <typename T>
int choose_bins(cblp_instance* h, hipStream_t s)
{
    h->bins_stale = false;
    h->H = h->Hb;
    h->H64 = h->Hb;
    if (sizeof(T) != 4 || h->n <= h->Hb || h->L == 0) return CBLP_OK;
    const int64_t Hc = std::min<int64_t>(h->n, h->bin_bytes / 4);
    const int G = h->seg_grid;
    unsigned long long* Ub = nullptr;
    int* dneed = nullptr;
    int rc;
    if ((rc = dalloc(&Ub, (size_t)Hc * G * 8))) return rc;
    if ((rc = dalloc(&dneed, sizeof(int)))) {
        (void)hipFree(Ub);
        return rc;
    }
    int need = 0;
    hipError_t e = hipMemsetAsync(Ub, 0, (size_t)Hc * G * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(dneed, 0, sizeof(int), s);
    if (e == hipSuccess)
        e = launch_bin_bound(h->L, h->pair_end, h->quad_end, G, h->ptr2, h->idx2, h->v2, h->den2,
                             h->vt0, h->lam2, h->fx_scale, (int)Hc, Ub, dneed, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&need, dneed, sizeof(int), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(Ub);
    (void)hipFree(dneed);
    if (e != hipSuccess || e2 != hipSuccess) return fail(CBLP_EHIP, "bin bound kernels failed");
    const int64_t H = std::min<int64_t>(h->n, (h->bin_bytes - 4 * (int64_t)need) / 4);
    if (H > h->Hb && H >= need) {
        h->H = (int)H;
        h->H64 = need;
    }
    return CBLP_OK;
}

template <typename T>
int run_segments(cblp_instance* h, void* seg_R, bool pseg, bool eval_out, hipStream_t s)
{
    int rc0;
    if (h->bins_stale && (rc0 = choose_bins<T>(h, s))) return rc0;
    SegArgs a;
    a.L = h->L;
    a.ptr = h->ptr2;
    a.idx = h->idx2;
    a.v = h->v2;
    a.den = h->den2;
    a.vt0 = h->vt0;
    a.lam = h->lam2;
    a.Rwarm = h->Rwarm;
    a.perm = h->perm;
    a.rho = h->rho;
    a.n = h->n;
    a.H = h->H;
    a.H64 = h->H64;
    a.hp = h->hp;
    a.S_fx = h->S_fx;
    a.brow = h->brow;
    a.row_words = h->row_words;
    a.fx_scale = h->fx_scale;
    a.zpart = h->zpart;
    a.z_scale = h->z_scale;
    a.z_rmax = h->z_rmax;
    a.seg_R = seg_R;
    a.seg_thr = eval_out ? h->eval_thr : nullptr;
    a.seg_lamD = eval_out ? h->eval_lamD : nullptr;
    a.psum = pseg ? h->psum : nullptr;
    a.rlib = h->rlib;
    a.inv_fx = 1.0 / h->fx_scale;
    a.psum_reset = h->psum_reset_next ? 1 : 0;
    a.woff = h->woff;
    a.idx3 = h->idx3;
    a.v3 = h->v3;
    a.den3 = h->den3;
    size_t slot;
    int rc = timed_begin(h, 0, s, &slot);
    if (rc) return rc;
    // views of the pair part [0, P2), the quad part [P2, P4) and the rest
    // (the FP64 kernels have only the 8-lane part: P2 = P4 = 0)
    const int64_t P2 = h->pair_end, P4 = h->quad_end;
    const size_t esz = h->esz;
    auto view = [&](int64_t p0, int64_t p1, int64_t wo) {
        SegArgs v = a;
        v.L = p1 - p0;
        v.ptr = h->ptr2 + p0;
        v.vt0 = (const char*)h->vt0 + p0 * esz;
        v.lam = (const char*)h->lam2 + p0 * esz;
        v.Rwarm = (char*)h->Rwarm + p0 * esz;
        v.perm = h->perm + p0;
        v.woff = h->woff + wo;
        if (v.seg_thr) {
            v.seg_thr = (char*)h->eval_thr + p0 * esz;
            v.seg_lamD = (char*)h->eval_lamD + p0 * esz;
        }
        if (v.psum) v.psum = h->psum + p0;
        return v;
    };
    const SegArgs a2 = view(0, P2, 0), a4 = view(P2, P4, h->woff_q),
                  a8 = view(P4, h->L, h->woff_b);
    HIP_TRY(launch_segments<T>(a2, a4, a8, h->seg_grid, h->seg_variant, pseg, s));
    h->fold_pending = true;
    return timed_end(h, slot, s);
}

template <typename T>
int run_phase(cblp_instance* h, void* eta, const spfom_params* p, int mode, double* row,
              hipStream_t s)
{
    PhaseArgs a;
    a.n = h->n;
    a.m = h->m;
    a.mode = mode;
    a.keep_sales = 0;
    a.rule = p ? p->rule : 0;
    a.check_every = p ? p->check_every : 1;
    a.gamma = p ? p->gamma : 1.0;
    a.mu = p ? p->mu : 0.0;
    a.tau_s = p ? p->tau : 1.0;
    a.tau_mult = tau_multiplier(p, h->t + 1);
    a.tau_vec = p ? p->tau_vec : nullptr;
    a.zpart = h->zpart;
    a.inv_z = 1.0 / h->z_scale;
    a.nz = h->seg_grid;
    a.S_fx = h->S_fx;
    a.inv_fx = 1.0 / h->fx_scale;
    a.r = h->r;
    a.c = h->c;
    a.a_ptr = h->a_ptr;
    a.a_idx = h->a_idx;
    a.a_val = h->a_val;
    a.at_ptr = h->at_ptr;
    a.at_prod = h->at_prod;
    a.at_val = h->at_val;
    a.eta = eta;
    a.rho = h->rho;
    a.S_d = h->S_d;
    a.u_d = h->u_d;
    a.sum_u = h->sum_u;
    a.bpart = h->bpart;
    a.bpart2 = h->bpart2;
    a.fold_blocks = h->fold_blocks;
    a.pnew = h->pnew;
    a.pinv = h->pinv;
    a.brow = h->brow;
    a.row_words = h->row_words;
    a.nrows = h->fold_pending ? h->seg_grid : 0;   // the segment pass's rows, added once
    a.rows_H = h->H;
    a.rows_H64 = h->H64;
    h->fold_pending = false;
    a.arrive = h->arrive;
    a.st = h->st;
    a.par = (int)(h->t & 1);
    a.row = row;
    if (mode == 2) {   // minibatch: the running totals, kept; no dual bound
        a.S_fx = h->mb_S;
        a.keep_sales = 1;
        a.nz = 0;
    }
    // the per-segment bound at a check of a window that accumulated psum
    const bool check = p && mode == 0 && (h->t + 1) % p->check_every == 0;
    const bool pseg = check && p->bound == SPFOM_BOUND_SEGMENT && h->pseg_window_ok;
    a.theta_prod = h->theta_prod;
    a.L = h->L;
    a.ptr2 = h->ptr2;
    a.idx2 = h->idx2;
    a.psum = h->psum;
    a.pseg_part = pseg ? h->pseg_part : nullptr;
    a.pseg_blocks = kPsegBlocks;
    size_t slot;
    int rc = timed_begin(h, 1, s, &slot);
    if (rc) return rc;
    HIP_TRY(launch_phase<T>(a, h->a_ptr == nullptr, s));
    return timed_end(h, slot, s);
}

template <typename T>
int iterate_impl(cblp_instance* h, void* eta, const spfom_params* p, int64_t iters,
                 bool keep_trace, hipStream_t s)
{
    const bool pseg = p->bound == SPFOM_BOUND_SEGMENT;
    int rc;
    if (pseg && (rc = ensure_pseg<T>(h, s))) return rc;
    HIP_TRY(launch_prices<T>(h->n, h->r, eta, h->a_ptr, h->a_idx, h->a_val, h->pnew, h->rho, s));
    for (int64_t it = 0; it < iters; ++it) {
        double* row = h->trace + (keep_trace ? it : 0) * SPFOM_NTRACE;
        if ((rc = run_segments<T>(h, nullptr, pseg, false, s))) return rc;
        if ((rc = run_phase<T>(h, eta, p, 0, row, s))) return rc;
        h->t += 1;
        // the averaging window restarts after t = 1 and whenever t doubles its
        // start (the device state does the same)
        const bool restart = h->t == 1 || h->t == 2 * h->t0h;
        if (restart) h->t0h = h->t;
        if (!pseg) h->pseg_window_ok = false;
        if (restart) h->pseg_window_ok = true;
        if (pseg) h->psum_reset_next = false;
        if (restart) h->psum_reset_next = true;
    }
    return CBLP_OK;
}

// Stochastic minibatch iterations: the sampled segments' pass, then the dual
// phase on the running sales totals (kept between iterations), dual step only.
template <typename T>
int minibatch_impl(cblp_instance* h, void* eta, const spfom_params* p, const int32_t* batch,
                   int64_t B, int64_t iters, bool keep_trace, hipStream_t s)
{
    int rc;
    if (!h->mb_S) {
        if ((rc = dalloc(&h->mb_ent, (size_t)std::max<int64_t>(h->nnz, 1) * mb_ent_bytes<T>())) ||
            (rc = dalloc(&h->mb_S, (size_t)h->n * 8)) ||
            (rc = dalloc(&h->mb_rec, (size_t)std::max<int64_t>(h->L, 1) * kMbRecBytes)) ||
            (rc = dalloc(&h->mb_stamp, (size_t)std::max<int64_t>(h->L, 1) * 4)) ||
            (rc = dalloc(&h->mb_err, sizeof(unsigned))))
            return rc;
        HIP_TRY(launch_minibatch_init(h->L, h->mb_stamp, s));
        h->mb_clear = true;
    }
    if (h->mb_clear) {   // y^0 = 0: the entries' kept sales and the totals
        HIP_TRY(hipMemsetAsync(h->mb_S, 0, (size_t)h->n * 8, s));
        HIP_TRY(launch_minibatch_records<T>(h->L, h->perm, h->ptr2, h->vt0, h->lam2, h->mb_rec,
                                            h->nnz, h->idx2, h->v2, h->den2, h->mb_ent, s));
        h->mb_clear = false;
    }
    HIP_TRY(hipMemsetAsync(h->mb_err, 0, sizeof(unsigned), s));
    HIP_TRY(launch_prices<T>(h->n, h->r, eta, h->a_ptr, h->a_idx, h->a_val, h->pnew, h->rho, s));
    MbArgs a;
    a.L = h->L;
    a.B = B;
    a.rec = h->mb_rec;
    a.ent = h->mb_ent;
    a.Rwarm = h->Rwarm;
    a.rho = h->rho;
    a.fx_scale = h->fx_scale;
    a.H = minibatch_bins<T>(h->n);
    a.S_run = h->mb_S;
    a.stamp = h->mb_stamp;
    a.err = h->mb_err;
    for (int64_t it = 0; it < iters; ++it) {
        a.batch = batch + it * B;
        a.it = h->mb_it;
        h->mb_it = h->mb_it == INT32_MAX ? 0 : h->mb_it + 1;
        HIP_TRY(launch_minibatch<T>(a, s));
        double* row = h->trace + (keep_trace ? it : 0) * SPFOM_NTRACE;
        if ((rc = run_phase<T>(h, eta, p, 2, row, s))) return rc;
        h->t += 1;
    }
    unsigned err = 0;
    HIP_TRY(hipMemcpyAsync(&err, h->mb_err, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err) {
        h->mb_clear = true;
        return fail(CBLP_EINVAL, (err & 1u) ? "batch holds a segment id outside [0, L)"
                                            : "batch lists a segment twice in one iteration");
    }
    return CBLP_OK;
}

template <typename T>
int evaluate_impl(cblp_instance* h, const void* eta, void* seg_R, double* s_out, hipStream_t s)
{
    int rc;
    if (s_out && !h->eval_thr) {
        const size_t bytes = (size_t)std::max<int64_t>(h->L, 1) * h->esz;
        if ((rc = dalloc(&h->eval_thr, bytes)) || (rc = dalloc(&h->eval_lamD, bytes))) return rc;
    }
    HIP_TRY(launch_prices<T>(h->n, h->r, eta, h->a_ptr, h->a_idx, h->a_val, h->pnew, h->rho, s));
    if ((rc = run_segments<T>(h, seg_R, false, s_out != nullptr, s))) return rc;
    if (s_out)
        HIP_TRY(launch_entry_sales<T>(h->L, h->perm, h->seg_ptr, h->idx, h->v, h->w, h->pnew,
                                      h->rho, h->eval_thr, h->eval_lamD, 1.0 / h->fx_scale, s_out,
                                      s));
    // evaluation leaves eta and the solver state untouched
    return run_phase<T>(h, const_cast<void*>(eta), nullptr, 1, h->trace, s);
}

int fill_stats(cblp_instance* h, spfom_stats* out, hipStream_t s, const double* dev_row)
{
    HIP_TRY(hipMemcpyAsync(h->pinned, dev_row, SPFOM_NTRACE * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    bool finite = true;
    for (int q = 0; q < SPFOM_NTRACE; ++q) finite = finite && std::isfinite(h->pinned[q]);
    if (out) {
        out->iters = h->t;
        std::memcpy(out->trace, h->pinned, sizeof(out->trace));
        out->status = finite ? CBLP_OK : CBLP_ENONFINITE;
    }
    if (!finite) return fail(CBLP_ENONFINITE, "non-finite value in the trace row");
    return CBLP_OK;
}

int reset_state(cblp_instance* h, hipStream_t s)
{
    DevState st[2];
    std::memset(st, 0, sizeof(st));
    st[0].dbest = st[1].dbest = INFINITY;
    HIP_TRY(hipMemcpyAsync(h->st, st, sizeof(st), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(h->sum_u, 0, (size_t)h->m * sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    h->t = 0;
    h->t0h = 0;
    h->psum_reset_next = true;
    h->pseg_window_ok = true;
    h->mb_clear = true;   // the minibatch sales restart from 0
    return CBLP_OK;
}

template <typename T>
int build_transpose(cblp_instance* h, const std::vector<int64_t>& hap, hipStream_t s)
{
    const int64_t nA = h->nnzA, n = h->n, m = h->m;
    std::vector<int32_t> ai((size_t)std::max<int64_t>(nA, 1));
    std::vector<T> avT((size_t)std::max<int64_t>(nA, 1));
    if (nA > 0) {
        HIP_TRY(hipMemcpyAsync(ai.data(), h->a_idx, nA * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(avT.data(), h->a_val, nA * sizeof(T), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    std::vector<int64_t> tp((size_t)m + 1, 0);
    for (int64_t q = 0; q < nA; ++q) tp[ai[q] + 1]++;
    for (int64_t i = 0; i < m; ++i) tp[i + 1] += tp[i];
    std::vector<int64_t> fillp(tp.begin(), tp.end() - 1);
    std::vector<int32_t> tprod((size_t)std::max<int64_t>(nA, 1));
    std::vector<double> tval((size_t)std::max<int64_t>(nA, 1));
    for (int64_t j = 0; j < n; ++j)      // products in increasing order: fixed sum order
        for (int64_t q = hap[j]; q < hap[j + 1]; ++q) {
            const int64_t dst = fillp[ai[q]]++;
            tprod[dst] = (int32_t)j;
            tval[dst] = (double)avT[q];
        }
    int rc;
    if ((rc = dalloc(&h->at_ptr, (m + 1) * sizeof(int64_t)))) return rc;
    if ((rc = dalloc(&h->at_prod, std::max<int64_t>(nA, 1) * sizeof(int32_t)))) return rc;
    if ((rc = dalloc(&h->at_val, std::max<int64_t>(nA, 1) * sizeof(double)))) return rc;
    HIP_TRY(hipMemcpyAsync(h->at_ptr, tp.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (nA > 0) {
        HIP_TRY(hipMemcpyAsync(h->at_prod, tprod.data(), nA * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->at_val, tval.data(), nA * sizeof(double), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return CBLP_OK;
}

template <typename T>
int create_impl(cblp_instance* h, hipStream_t s)
{
    int rc;
    std::vector<int64_t> hap;
    const bool ident = h->a_ptr == nullptr;
    if (!ident) {
        hap.resize((size_t)h->n + 1);
        HIP_TRY(hipMemcpyAsync(hap.data(), h->a_ptr, (h->n + 1) * sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        h->nnzA = hap[h->n];
        if (h->nnzA < 0) return fail(CBLP_EINVAL, "a_ptr[n] < 0");
    }
    // validation on the device
    unsigned* dflags = nullptr;
    if ((rc = dalloc(&dflags, sizeof(unsigned)))) return rc;
    unsigned flags = 0;
    hipError_t e0 = hipMemsetAsync(dflags, 0, sizeof(unsigned), s);
    hipError_t e1 = e0 == hipSuccess
                        ? launch_validate<T>(h->L, h->n, h->m, h->nnz, h->nnzA, h->seg_ptr, h->idx,
                                             h->v, h->w, h->v0, h->lam, h->r, h->c, h->a_ptr,
                                             h->a_idx, h->a_val, dflags, s)
                        : e0;
    hipError_t e2 = e1 == hipSuccess
                        ? hipMemcpyAsync(&flags, dflags, sizeof(unsigned), hipMemcpyDeviceToHost, s)
                        : e1;
    hipError_t e3 = hipStreamSynchronize(s);
    (void)hipFree(dflags);
    if (e2 != hipSuccess || e3 != hipSuccess) return fail(CBLP_EHIP, "validation kernel failed");
    if (flags) {
        return fail(CBLP_EINVAL, cblp::validation_message(flags));
    }

    // launch shape: every resident 1024-thread segment block of every CU, each
    // with H LDS bins; blocks stride over tiles of 64 segments
    int cus = 256;
    size_t lds_block = 64 * 1024;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
        if (prop.multiProcessorCount > 0) cus = prop.multiProcessorCount;
        if (prop.sharedMemPerBlock > 0) lds_block = prop.sharedMemPerBlock;
    }
    // row pointers on the host: the longest row picks the register slots, and
    // the size-sorted copy below is built from them
    std::vector<int64_t> sp((size_t)h->L + 1);
    HIP_TRY(hipMemcpyAsync(sp.data(), h->seg_ptr, (h->L + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t kmax = 0;
    for (int64_t l = 0; l < h->L; ++l) kmax = std::max(kmax, sp[l + 1] - sp[l]);

    // The kernel follows from the dtype and the shape.  FP32: rows of at most
    // kPairMaxRow entries go to 2-lane groups, of at most kQuadMaxRow to
    // 4-lane groups, longer ones to 8-lane groups; the prices go to LDS when
    // they take at most half of it, else the popular head of them does.
    // FP64: 8-lane groups with the prices in global memory.  Product ids are
    // stored in 16 bits when they fit.
    const bool prices_fit = (int64_t)h->n * (int64_t)sizeof(T) * 2 <= (int64_t)lds_block;
    const bool ids16 = h->n <= 65536;
    if (sizeof(T) == 4)
        h->seg_variant = (prices_fit && ids16) ? kSegMixed3
                         : ids16 ? kSegMixed3Split16 : kSegMixed3Split32;
    else
        h->seg_variant = ids16 ? kSegSlots16 : kSegSlots32;
    h->idx16 = seg_idx16(h->seg_variant);
    h->hp = seg_split(h->seg_variant) ? (int)std::min<int64_t>(h->n, kSplitPrices) : 0;
    const int64_t price_bytes = seg_split(h->seg_variant) ? (int64_t)h->hp * (int64_t)sizeof(T)
                                : seg_lds_prices(h->seg_variant) ? h->n * (int64_t)sizeof(T) : 0;
    h->bin_bytes = ((int64_t)lds_block - 1024 - price_bytes) & ~(int64_t)7;
    // 64-bit bins for the most popular products; the FP32 segment kernel may
    // trade them for more 32-bit ones once the values are known (choose_bins)
    h->Hb = (int)std::max<int64_t>(1, std::min<int64_t>({h->n, (int64_t)kMaxBins, h->bin_bytes / 8}));
    h->H = h->Hb;
    h->H64 = h->Hb;
    h->bins_stale = true;
    const int per_cu = segment_blocks_per_cu<T>(h->H, h->H64, h->n, h->hp, h->seg_variant);
    const int64_t tiles = (h->L + kSegsPerTile - 1) / kSegsPerTile;
    h->seg_grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cus * per_cu));
    h->fold_blocks = (int)((h->n + kFoldLite - 1) / kFoldLite);
    const int64_t row_blocks = (h->m + kRowThreads - 1) / kRowThreads;

    const size_t esz = h->esz;
    const int64_t L1 = std::max<int64_t>(h->L, 1);
    if ((rc = dalloc(&h->rho, (size_t)h->n * esz))) return rc;
    if ((rc = dalloc(&h->S_fx, (size_t)h->n * 8))) return rc;
    if ((rc = dalloc(&h->S_d, (size_t)h->n * 8))) return rc;
    if ((rc = dalloc(&h->u_d, (size_t)h->m * 8))) return rc;
    if ((rc = dalloc(&h->sum_u, (size_t)h->m * 8))) return rc;
    // fold partials: one per 256 products, or per 64 in the fused step
    if ((rc = dalloc(&h->bpart, (size_t)((h->n + 63) / 64 + 1) * 8 * 8))) return rc;
    if ((rc = dalloc(&h->bpart2, (size_t)std::max<int64_t>(row_blocks, 1) * 8 * 8))) return rc;
    if ((rc = dalloc(&h->st, 2 * sizeof(DevState)))) return rc;
    if ((rc = dalloc(&h->arrive, sizeof(unsigned)))) return rc;
    HIP_TRY(hipMemsetAsync(h->arrive, 0, sizeof(unsigned), s));   // the last block resets it
    if ((rc = ensure_trace(h, 64))) return rc;
    if (hipHostMalloc((void**)&h->pinned, SPFOM_NTRACE * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return fail(CBLP_ENOMEM, "hipHostMalloc failed");

    // product ids by falling degree (ties keep their order), unless the
    // caller's numbering already is that order
    {
        if (h->n > 1 && h->nnz > 0) {
            unsigned long long* ddeg = nullptr;
            if ((rc = dalloc(&ddeg, (size_t)h->n * 8))) return rc;
            std::vector<unsigned long long> deg((size_t)h->n);
            hipError_t d1 = launch_degree(h->nnz, h->idx, h->n, ddeg, s);
            hipError_t d2 = d1 == hipSuccess ? hipMemcpyAsync(deg.data(), ddeg, (size_t)h->n * 8,
                                                              hipMemcpyDeviceToHost, s)
                                             : d1;
            hipError_t d3 = hipStreamSynchronize(s);
            (void)hipFree(ddeg);
            if (d2 != hipSuccess || d3 != hipSuccess) return fail(CBLP_EHIP, "degree kernel failed");
            bool sorted = true;
            for (int64_t j = 1; j < h->n && sorted; ++j) sorted = deg[j] <= deg[j - 1];
            if (!sorted) {
                std::vector<int32_t> order((size_t)h->n), pnew((size_t)h->n);
                for (int64_t j = 0; j < h->n; ++j) order[j] = (int32_t)j;
                std::stable_sort(order.begin(), order.end(),
                                 [&](int32_t x, int32_t y) { return deg[x] > deg[y]; });
                for (int64_t q = 0; q < h->n; ++q) pnew[order[q]] = (int32_t)q;
                if ((rc = dalloc(&h->pnew, (size_t)h->n * 4))) return rc;
                if ((rc = dalloc(&h->pinv, (size_t)h->n * 4))) return rc;
                HIP_TRY(hipMemcpyAsync(h->pnew, pnew.data(), (size_t)h->n * 4,
                                       hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync(h->pinv, order.data(), (size_t)h->n * 4,
                                       hipMemcpyHostToDevice, s));
                HIP_TRY(hipStreamSynchronize(s));
            }
        }
    }

    // size-sorted copy of the segments: a stable counting sort by row length
    {
        std::vector<int64_t> start((size_t)kmax + 2, 0);
        for (int64_t l = 0; l < h->L; ++l) start[sp[l + 1] - sp[l] + 1]++;
        for (int64_t k = 0; k <= kmax; ++k) start[k + 1] += start[k];
        std::vector<int32_t> perm((size_t)L1, 0);
        for (int64_t l = 0; l < h->L; ++l) perm[start[sp[l + 1] - sp[l]]++] = (int32_t)l;
        std::vector<int64_t> ptr((size_t)h->L + 1, 0);
        for (int64_t p = 0; p < h->L; ++p) ptr[p + 1] = ptr[p] + (sp[perm[p] + 1] - sp[perm[p]]);
        if ((rc = dalloc(&h->ptr2, (size_t)(h->L + 1) * 8))) return rc;
        if ((rc = dalloc(&h->perm, (size_t)L1 * 4))) return rc;
        // the copy is followed by kPad entries (product 0, v = 0, den = 1)
        const size_t ne = (size_t)h->nnz + kPad;
        if ((rc = dalloc(&h->idx2, ne * 4))) return rc;
        if ((rc = dalloc(&h->v2, ne * esz))) return rc;
        if ((rc = dalloc(&h->den2, ne * esz))) return rc;
        HIP_TRY(hipMemsetAsync(h->idx2 + h->nnz, 0, kPad * 4, s));
        HIP_TRY(hipMemsetAsync((char*)h->v2 + h->nnz * esz, 0, kPad * esz, s));
        {
            std::vector<T> ones(kPad, T(1));
            HIP_TRY(hipMemcpyAsync((char*)h->den2 + h->nnz * esz, ones.data(), kPad * esz,
                                   hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        if ((rc = dalloc(&h->vt0, (size_t)L1 * esz))) return rc;
        if ((rc = dalloc(&h->lam2, (size_t)L1 * esz))) return rc;
        if ((rc = dalloc(&h->Rwarm, (size_t)L1 * esz))) return rc;
        if ((rc = dalloc(&h->v0c, (size_t)L1 * esz))) return rc;
        HIP_TRY(hipMemcpyAsync(h->ptr2, ptr.data(), (h->L + 1) * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(h->perm, perm.data(), L1 * 4, hipMemcpyHostToDevice, s));
        if (h->L > 0)
            HIP_TRY(launch_relayout<T>(h->L, h->seg_ptr, h->idx, h->v, h->w, h->v0, h->lam,
                                       h->perm, h->pnew, h->ptr2, h->idx2, h->v2, h->den2, h->vt0,
                                       h->lam2, h->Rwarm, h->v0c, s));
        {
            // slot-major copy: wave-tile w of a part (positions Rw..Rw+R-1 of
            // it, R = 64 / G rows of G lanes) gets 64 entries per slot for as
            // many slots as its longest row needs (at least one).  FP32:
            // positions [0, P2) (rows of at most kPairMaxRow entries; rows
            // ascend) in the pair layout, [P2, P) (at most kQuadMaxRow) in the
            // quad layout, the rest in the 8-lane one, each part with its own
            // offsets (one spare entry each).  Part boundaries are rounded down
            // to multiples of kPartAlign positions, so that every part starts
            // on a tile of every layout; a row just below a boundary goes to
            // the wider groups.  FP64: one 8-lane part.
            const bool mixed3 = seg_mixed3(h->seg_variant);
            int64_t P2 = 0, P = 0;
            if (mixed3) {
                while (P2 < h->L && ptr[P2 + 1] - ptr[P2] <= kPairMaxRow) ++P2;
                P = P2;
                while (P < h->L && ptr[P + 1] - ptr[P] <= kQuadMaxRow) ++P;
                P2 = P2 / kPartAlign * kPartAlign;
                P = P / kPartAlign * kPartAlign;
            }
            h->pair_end = P2;
            h->quad_end = P;
            std::vector<int64_t> woff;
            auto part = [&](int64_t p0, int64_t p1, int64_t G) {
                const int64_t R = 64 / G, W = (p1 - p0 + R - 1) / R;
                const size_t w0 = woff.size();
                woff.push_back(w0 == 0 ? 0 : woff.back());
                for (int64_t w = 0; w < W; ++w) {
                    int64_t kw = 0;
                    for (int64_t p = p0 + w * R; p < std::min(p1, p0 + (w + 1) * R); ++p)
                        kw = std::max(kw, ptr[p + 1] - ptr[p]);
                    woff.push_back(woff.back() + 64 * std::max<int64_t>(1, (kw + G - 1) / G));
                }
                woff.push_back(woff.back());
                return w0;
            };
            part(0, P2, 2);
            h->woff_q = (int64_t)part(P2, P, 4);
            h->woff_b = (int64_t)part(P, h->L, kGroup);
            const int64_t entries = woff.back() + 64 * kMaxJ;   // loads may run J slots past the end
            h->slot_entries = woff.back();
            if ((rc = dalloc(&h->woff, woff.size() * 8))) return rc;
            if ((rc = dalloc(&h->idx3, (size_t)entries * (h->idx16 ? 2 : 4)))) return rc;
            if ((rc = dalloc(&h->v3, (size_t)entries * esz))) return rc;
            if ((rc = dalloc(&h->den3, (size_t)entries * esz))) return rc;
            HIP_TRY(hipMemcpyAsync(h->woff, woff.data(), woff.size() * 8, hipMemcpyHostToDevice, s));
            HIP_TRY(launch_relayout_slots<T>(P2, h->ptr2, h->idx2, h->v2, h->den2, h->woff,
                                             entries, h->idx3, h->idx16, 2, h->v3, h->den3, s));
            HIP_TRY(launch_relayout_slots<T>(P - P2, h->ptr2 + P2, h->idx2, h->v2, h->den2,
                                             h->woff + h->woff_q, 0, h->idx3, h->idx16, 4,
                                             h->v3, h->den3, s));
            HIP_TRY(launch_relayout_slots<T>(h->L - P, h->ptr2 + P, h->idx2, h->v2, h->den2,
                                             h->woff + h->woff_b, 0, h->idx3, h->idx16, kGroup,
                                             h->v3, h->den3, s));
        }
        HIP_TRY(hipStreamSynchronize(s));   // the host vectors die here
    }
    if ((rc = dalloc(&h->zpart, (size_t)h->seg_grid * 8))) return rc;
    // one row of bins per segment block, as long as the largest layout
    h->row_words = (h->bin_bytes + 255) / 256 * 32;
    if ((rc = dalloc(&h->brow, (size_t)h->seg_grid * (size_t)h->row_words * 8))) return rc;

    // fixed-point scale of the sales sums from the arrival rates
    const int pblocks = 256;
    double* lp = nullptr;
    if ((rc = dalloc(&lp, 2 * pblocks * sizeof(double)))) return rc;
    std::vector<double> hl(2 * pblocks);
    hipError_t p1 = launch_prepare<T>(h->L, h->lam, lp, pblocks, s);
    hipError_t p2 = p1 == hipSuccess
                        ? hipMemcpyAsync(hl.data(), lp, 2 * pblocks * sizeof(double), hipMemcpyDeviceToHost, s)
                        : p1;
    hipError_t p3 = hipStreamSynchronize(s);
    (void)hipFree(lp);
    if (p2 != hipSuccess || p3 != hipSuccess) return fail(CBLP_EHIP, "prepare kernel failed");
    double tot = 0.0, hi = 0.0;
    for (int q = 0; q < pblocks; ++q) {
        tot += hl[2 * q];
        hi = std::max(hi, hl[2 * q + 1]);
    }
    // every 64-bit sum stays below 2^61; an FP32 quantum below 2^30
    int e_tot = 0, e_hi = 0;
    std::frexp(tot + 1.0, &e_tot);
    std::frexp(hi, &e_hi);
    int bits = std::min(60, 61 - e_tot);
    if (h->dtype == CBLP_F32) bits = std::min(bits, 30 - e_hi);
    if (bits < 8) return fail(CBLP_EINVAL, "arrival rates too large for the fixed-point sales sums");
    h->fx_scale = std::ldexp(1.0, bits);

    // fixed-point scale of Z = sum lambda R*: with duals >= 0, R* <= max r, so
    // sum lambda max(r) (1 + 2^-20) 2^zb stays below 2^60
    {
        std::vector<T> hr((size_t)h->n);
        HIP_TRY(hipMemcpyAsync(hr.data(), h->r, (size_t)h->n * sizeof(T), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double rmax = 0.0;
        for (const T x : hr) rmax = std::max(rmax, (double)x);
        h->z_rmax = rmax * (1.0 + std::ldexp(1.0, -20));
        int e_z = 0;
        std::frexp(tot * h->z_rmax + 1.0, &e_z);
        const int zb = std::min(60, 60 - e_z);
        if (zb < 0) return fail(CBLP_EINVAL, "arrival rates times revenues too large for the fixed-point dual bound");
        h->z_scale = std::ldexp(1.0, zb);
    }

    if (!ident && (rc = build_transpose<T>(h, hap, s))) return rc;

    HIP_TRY(hipMemsetAsync(h->S_fx, 0, (size_t)h->n * 8, s));
    return reset_state(h, s);
}

}  // namespace

std::string cblp::validation_message(unsigned flags)
{
    std::string msg = "invalid instance:";
    for (int b = 0; b < V_NBITS; ++b)
        if (flags & (1u << b)) msg += std::string(" ") + kValidationText[b] + ";";
    return msg;
}

int cblp::reset_handle_state(cblp_instance* h, hipStream_t s) { return reset_state(h, s); }

int cblp::refresh_launch(cblp_instance* h, unsigned* flags, hipStream_t s)
{
    HIP_TRY(h->dtype == CBLP_F32 ? launch_refresh<float>(h, flags, s)
                                 : launch_refresh<double>(h, flags, s));
    h->mb_clear = true;
    h->bins_stale = true;   // the bin bounds follow the values
    return CBLP_OK;
}

extern "C" {

const char* cblp_last_error(void) { return g_err.c_str(); }

int cblp_create(cblp_t* out, int64_t L, int64_t n, int64_t m, const int64_t* seg_ptr,
                const int32_t* prod_idx, const void* v, const void* w, const void* v0,
                const void* lambda, const void* r, const int64_t* a_ptr, const int32_t* a_idx,
                const void* a_val, const void* c, int32_t dtype, void* stream)
{
    g_err.clear();
    if (!out) return fail(CBLP_EINVAL, "out is NULL");
    *out = nullptr;
    if (L < 0 || n <= 0 || m <= 0) return fail(CBLP_EINVAL, "need L >= 0, n > 0, m > 0");
    if (n > INT32_MAX || m > INT32_MAX) return fail(CBLP_EINVAL, "n and m must fit in int32");
    if (dtype != CBLP_F32 && dtype != CBLP_F64)
        return fail(CBLP_EINVAL, "dtype must be CBLP_F32 or CBLP_F64");
    if (!seg_ptr || !r || !c || (L > 0 && (!v0 || !lambda)))
        return fail(CBLP_EINVAL, "NULL instance array");
    const bool ident = !a_ptr && !a_idx && !a_val;
    if (!ident && (!a_ptr || !a_idx || !a_val))
        return fail(CBLP_EINVAL, "a_ptr, a_idx, a_val must be all NULL or all set");
    if (ident && m != n) return fail(CBLP_EINVAL, "identity resource matrix needs m == n");
    hipStream_t s = S(stream);

    cblp_instance* h = new (std::nothrow) cblp_instance();
    if (!h) return fail(CBLP_ENOMEM, "host allocation failed");
    if (hipGetDevice(&h->device) != hipSuccess) {
        release(h);
        return fail(CBLP_EHIP, "hipGetDevice failed");
    }
    h->dtype = dtype;
    h->esz = dtype == CBLP_F32 ? 4 : 8;
    h->L = L;
    h->n = n;
    h->m = m;
    h->seg_ptr = seg_ptr;
    h->idx = prod_idx;
    h->v = v;
    h->w = w;
    h->v0 = v0;
    h->lam = lambda;
    h->r = r;
    h->c = c;
    h->a_ptr = a_ptr;
    h->a_idx = a_idx;
    h->a_val = a_val;
    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, seg_ptr + L, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        release(h);
        return fail(CBLP_EHIP, "reading seg_ptr[L] failed");
    }
    if (nnz < 0 || (nnz > 0 && (!prod_idx || !v || !w))) {
        release(h);
        return fail(CBLP_EINVAL, "seg_ptr[L] < 0 or NULL CSR array");
    }
    h->nnz = nnz;
    const int rc = dtype == CBLP_F32 ? create_impl<float>(h, s) : create_impl<double>(h, s);
    if (rc) {
        release(h);
        return rc;
    }
    *out = h;
    return CBLP_OK;
}

void cblp_destroy(cblp_t h) { release(h); }

int cblp_refresh(cblp_t h, void* stream)
{
    g_err.clear();
    if (!h) return fail(CBLP_EINVAL, "handle is NULL");
    hipStream_t s = S(stream);
    unsigned* dflags = nullptr;
    int rc;
    if ((rc = dalloc(&dflags, sizeof(unsigned)))) return rc;
    unsigned flags = 0;
    hipError_t e0 = hipMemsetAsync(dflags, 0, sizeof(unsigned), s);
    rc = e0 == hipSuccess ? refresh_launch(h, dflags, s) : fail(CBLP_EHIP, "hipMemsetAsync failed");
    hipError_t e1 = rc == CBLP_OK ? hipMemcpyAsync(&flags, dflags, sizeof(unsigned),
                                                   hipMemcpyDeviceToHost, s)
                                  : hipSuccess;
    hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(dflags);
    if (rc) return rc;
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(CBLP_EHIP, "refresh kernel failed");
    if (flags) return fail(CBLP_EINVAL, validation_message(flags));
    return reset_state(h, s);
}

int spfom_reset(cblp_t h, void* stream)
{
    g_err.clear();
    if (!h) return fail(CBLP_EINVAL, "handle is NULL");
    return reset_state(h, S(stream));
}

int spfom_iterate(cblp_t h, void* eta, const spfom_params* p, int64_t iters, double* trace,
                  spfom_stats* out, void* stream)
{
    g_err.clear();
    if (!h || !eta) return fail(CBLP_EINVAL, "NULL handle or eta");
    if (iters < 0) return fail(CBLP_EINVAL, "iters < 0");
    int rc = check_params(p);
    if (rc) return rc;
    hipStream_t s = S(stream);
    if (trace && (rc = ensure_trace(h, std::max<int64_t>(iters, 1)))) return rc;
    if (iters == 0) {
        if (out) {
            std::memset(out, 0, sizeof(*out));
            out->iters = h->t;
        }
        return CBLP_OK;
    }
    rc = h->dtype == CBLP_F32 ? iterate_impl<float>(h, eta, p, iters, trace != nullptr, s)
                              : iterate_impl<double>(h, eta, p, iters, trace != nullptr, s);
    if (rc) return rc;
    if (trace) {
        HIP_TRY(hipMemcpyAsync(trace, h->trace, iters * SPFOM_NTRACE * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (out || trace) {
        const double* last = h->trace + (trace ? (iters - 1) * SPFOM_NTRACE : 0);
        rc = fill_stats(h, out, s, last);
        if (out) out->seconds = 0.0;
        return rc;
    }
    return CBLP_OK;
}

int spfom_minibatch(cblp_t h, void* eta, const spfom_params* p, const int32_t* batch, int64_t B,
                    int64_t iters, double* trace, void* stream)
{
    g_err.clear();
    if (!h || !eta || (!batch && iters > 0)) return fail(CBLP_EINVAL, "NULL handle, eta or batch");
    if (iters < 0) return fail(CBLP_EINVAL, "iters < 0");
    if (B < 1 || B > h->L) return fail(CBLP_EINVAL, "need 1 <= B <= L");
    int rc = check_params(p);
    if (rc) return rc;
    if (p->rule != SPFOM_STEP_CONST || (p->tau_decay > 0.0 && p->tau_decay < 1.0))
        return fail(CBLP_EINVAL, "minibatch iterations take the constant step");
    if (iters == 0) return CBLP_OK;
    hipStream_t s = S(stream);
    if (trace && (rc = ensure_trace(h, iters))) return rc;
    rc = h->dtype == CBLP_F32 ? minibatch_impl<float>(h, eta, p, batch, B, iters, trace != nullptr, s)
                              : minibatch_impl<double>(h, eta, p, batch, B, iters, trace != nullptr, s);
    if (rc) return rc;
    if (trace) {
        HIP_TRY(hipMemcpyAsync(trace, h->trace, iters * SPFOM_NTRACE * sizeof(double),
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return CBLP_OK;
}

int spfom_solve(cblp_t h, void* eta, const spfom_params* p, spfom_stats* out, void* stream)
{
    g_err.clear();
    if (!h || !eta || !out) return fail(CBLP_EINVAL, "NULL handle, eta or out");
    int rc = check_params(p);
    if (rc) return rc;
    if (p->max_iters < 0 || !(p->tol >= 0.0))
        return fail(CBLP_EINVAL, "need max_iters >= 0 and tol >= 0");
    hipStream_t s = S(stream);
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = reset_state(h, s))) return rc;
    std::memset(out, 0, sizeof(*out));
    out->status = CBLP_ENOTCONVERGED;
    while (h->t < p->max_iters) {
        const int64_t k = std::min<int64_t>(p->check_every, p->max_iters - h->t);
        rc = h->dtype == CBLP_F32 ? iterate_impl<float>(h, eta, p, k, false, s)
                                  : iterate_impl<double>(h, eta, p, k, false, s);
        if (rc) return rc;
        rc = fill_stats(h, out, s, h->trace);
        if (rc) {
            out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            return rc;
        }
        if (h->t % p->check_every == 0 && out->trace[SPFOM_TR_GAP] <= p->tol) {
            out->status = CBLP_OK;
            break;
        }
        out->status = CBLP_ENOTCONVERGED;
    }
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out->status != CBLP_OK)
        return fail(CBLP_ENOTCONVERGED, "certified gap above tol after max_iters iterations");
    return CBLP_OK;
}

int cblp_gap(cblp_t h, const void* eta, spfom_stats* out, void* stream)
{
    g_err.clear();
    if (!h || !eta || !out) return fail(CBLP_EINVAL, "NULL handle, eta or out");
    hipStream_t s = S(stream);
    int rc = h->dtype == CBLP_F32 ? evaluate_impl<float>(h, eta, nullptr, nullptr, s)
                                  : evaluate_impl<double>(h, eta, nullptr, nullptr, s);
    if (rc) return rc;
    rc = fill_stats(h, out, s, h->trace);
    out->seconds = 0.0;
    return rc;
}

int cblp_sales(cblp_t h, const void* eta, double* S_out, double* u_out, void* seg_R_out,
               double* s_out, void* stream)
{
    g_err.clear();
    if (!h || !eta) return fail(CBLP_EINVAL, "NULL handle or eta");
    hipStream_t s = S(stream);
    int rc = h->dtype == CBLP_F32 ? evaluate_impl<float>(h, eta, seg_R_out, s_out, s)
                                  : evaluate_impl<double>(h, eta, seg_R_out, s_out, s);
    if (rc) return rc;
    if (S_out) HIP_TRY(hipMemcpyAsync(S_out, h->S_d, h->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (u_out) HIP_TRY(hipMemcpyAsync(u_out, h->u_d, h->m * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CBLP_OK;
}

int cblp_launch_info(cblp_t h, int32_t* seg_grid, int32_t* bins, int32_t* bins64,
                     int32_t* fx_bits, int32_t* kernel, int64_t* slot_entries)
{
    g_err.clear();
    if (!h) return fail(CBLP_EINVAL, "handle is NULL");
    if (seg_grid) *seg_grid = h->seg_grid;
    if (bins) *bins = h->H;
    if (bins64) *bins64 = h->H64;
    if (fx_bits) {
        int e = 0;
        std::frexp(h->fx_scale, &e);
        *fx_bits = e - 1;
    }
    if (kernel) *kernel = h->seg_variant;
    if (slot_entries) *slot_entries = h->slot_entries;
    return CBLP_OK;
}

int cblp_timing(cblp_t h, int32_t enable)
{
    g_err.clear();
    if (!h) return fail(CBLP_EINVAL, "handle is NULL");
    h->timing = enable != 0;
    h->ev_used = 0;
    h->ev_marks.clear();
    return CBLP_OK;
}

int cblp_timing_read(cblp_t h, double* ms, int64_t* launches, void* stream)
{
    g_err.clear();
    if (!h || !ms || !launches) return fail(CBLP_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(S(stream)));
    ms[0] = ms[1] = 0.0;
    launches[0] = launches[1] = 0;
    for (const auto& mk : h->ev_marks) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, h->ev_pool[mk.second], h->ev_pool[mk.second + 1]));
        ms[mk.first] += (double)t;
        launches[mk.first] += 1;
    }
    h->ev_used = 0;
    h->ev_marks.clear();
    return CBLP_OK;
}

}  // extern "C"

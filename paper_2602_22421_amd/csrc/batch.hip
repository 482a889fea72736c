// Batched re-solves: many independent CBLP instances - the per-period
// re-solves of the multi-period setting of Section 5.1, each with its
// remaining capacities - advance together.  One iteration for all of them is
// one persistent segment launch and two dual-phase launches; spfom_batch_solve
// replays check_every iterations from a hipGraph and drops converged
// instances between replays.
//
// Work list.  Each instance's size-sorted tiles (128 positions) are cut into
// work items of about the same size; items are ordered largest instance first
// and handed out through an atomic counter, so large and small instances share
// the machine without a static schedule.  An item adds its LDS bins to its
// instance's 64-bit sales sums with integer atomics and writes its own
// fixed-point partial of sum lambda R*, so the results do not depend on which
// block ran which item.
//
// Dual phase.  Fold blocks (64 products of one instance) and row blocks (256
// rows of one instance) come from flattened tables; every row block of an
// instance folds that instance's partials in the same order (no fences) and
// the one at row 0 writes the instance's next state and trace row.  The state
// is double-buffered per instance: the copy with the larger iteration count is
// current, the other is written.
//
// Scope: identity resource matrix (m == n) for every instance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <cstdio>
#include <string>
#include <vector>

#include "dual_core.hpp"
#include "handle.hpp"
#include "segment_core.hpp"

namespace cblp {
namespace {

struct BInst {
    SegArgs seg;               // this instance's sorted copy and tail accumulator
    SegArgs part_args[3];           // its pair, quad and 8-lane parts (slot-major copies),
    int64_t pstart[3];         // each viewed from its first position pstart[k]
    int64_t n, m;
    const void* r;
    const void* c;
    void* eta;
    void* rho;
    const void* tau_vec;
    double tau_s;
    unsigned long long* S_fx;
    double inv_fx;
    double inv_z;              // 1 / the Z fixed-point scale
    double* S_d;
    double* u_d;
    double* sum_u;
    DevState* st;              // [2]
    double* row;               // [SPFOM_NTRACE]
    int item0, item1;          // work items of this instance
    int fold0, fold1;          // its fold blocks
    int H;                     // LDS bins (library products [0, H))
    int active;
    const int32_t* pnew;       // [n] library id of caller product j; NULL: j
    const int32_t* pinv;       // [n] caller product of library id q; NULL: q
};

struct BItem {
    int inst;
    int part;                  // 0 pair, 1 quad, 2 8-lane part of the slot-major copy
    int64_t p0, p1;            // positions [p0, p1) (p0 on a block tile of the part's layout)
};

struct BChunk {
    int inst;
    int pad;
    int64_t j0;                // first product (fold) or row (update)
};

struct BArgs {
    const BInst* inst;
    const BChunk* fold;
    const BChunk* rows;
    const long long* zpart;    // fixed-point Z partials per item
    double* bpart;             // [fold blocks][8]
    int rule, check_every;
    double gamma, mu;
    double tau_decay;          // CONST: step tau * tau_decay^k in iterations kE+1..(k+1)E
    long long decay_every;     // E
    unsigned* counter;         // the segment kernel's work counter, cleared by k_bfold
};

// the fields row_work reads, for one instance
struct RowView {
    const void* c;
    const void* eta;
    const void* tau_vec;
    double tau_s;
    double* u_d;
    double* sum_u;
    int mode;
};

__device__ __forceinline__ int current(const DevState* st) { return st[0].t >= st[1].t ? 0 : 1; }


// MODE 0: prices gathered from global memory; 1: the item's instance prices
// copied into LDS behind the largest instance's bins (Hmax), then gathered
// there; 3: as 1 over the handles' own slot-major copies, each part by the
// groups of its width (2, 4 or 8 lanes; FP32, else 8 lanes only; IdxT: the
// copies' product id type).
template <typename T, int J, int DEPTH, int MODE, typename IdxT = int32_t>
__global__ void __launch_bounds__(kSegThreads)
k_bsegments(const BInst* __restrict__ inst, const BItem* __restrict__ items, int nitems, unsigned* counter,
            long long* zpart, int Hmax)
{
    extern __shared__ unsigned long long bins[];
    __shared__ long long zsh[kSegThreads / 64];
    __shared__ int s_item;
    T* lprice = (T*)(bins + Hmax);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        // the item is block-uniform: keep it (and the instance record) in SGPRs
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= nitems) break;
        const BItem w = items[it];
        const BInst* I = inst + w.inst;
        if (!I->active) continue;
        const SegArgs a = I->seg;
        const int H = a.H;
        for (int j = threadIdx.x; j < H; j += kSegThreads) bins[j] = 0ull;
        if (MODE > 0)
            for (int64_t j = threadIdx.x; j < a.n; j += kSegThreads) lprice[j] = ((const T*)a.rho)[j];
        __syncthreads();
        ZAcc zacc;
        const seg::FlatPrices<T> pr{MODE > 0 ? (const T*)lprice : (const T*)a.rho};
        const int64_t t0 = w.p0 / kSegsPerTile, t1 = (w.p1 + kSegsPerTile - 1) / kSegsPerTile;
        if constexpr (MODE == 3) {
            const SegArgs& ap = I->part_args[w.part];   // fields read where used: fewer live registers
            const int64_t q0 = w.p0 - I->pstart[w.part], q1 = w.p1 - I->pstart[w.part];
            bool done = false;
            if constexpr (sizeof(T) == 4) {
                if (w.part == 0) {
                    seg::process_tiles_pair<T, 8, seg::FlatPrices<T>, IdxT>(
                        ap, q0 / seg::kPairTileRows,
                        (q1 + seg::kPairTileRows - 1) / seg::kPairTileRows, 1, bins, pr, zacc);
                    done = true;
                } else if (w.part == 1) {
                    seg::process_tiles_quad<T, 8, seg::FlatPrices<T>, IdxT>(
                        ap, q0 / seg::kQuadTileRows,
                        (q1 + seg::kQuadTileRows - 1) / seg::kQuadTileRows, 1, bins, pr, zacc);
                    done = true;
                }
            }
            if (!done)   // the 8-lane part (FP64 handles have no other)
                seg::process_tiles_slots<T, J, false, seg::FlatPrices<T>, IdxT>(
                    ap, q0 / kSegsPerTile, (q1 + kSegsPerTile - 1) / kSegsPerTile, 1, bins, pr,
                    zacc);
        } else {
            seg::process_tiles<T, J, DEPTH>(a, t0, t1, 1, bins, pr, zacc);
        }
        __syncthreads();
        // the item's bins into the instance's 64-bit sales sums: integer adds,
        // so the sums do not depend on which block ran which item
        for (int j = threadIdx.x; j < H; j += kSegThreads)
            if (bins[j]) atomicAdd(&I->S_fx[j], bins[j]);
        const long long z = block_z(zacc, zsh);
        if (threadIdx.x == 0) zpart[it] = z;
    }
}

template <typename T>
// One wave per fold block: thread jj owns library product j0 + jj (caller
// product pinv[j0 + jj]); the single instance's fold takes the same
// per-product values through the same wave reduction.
__global__ void __launch_bounds__(kFoldProducts) k_bfold(BArgs b)
{
    using namespace dual;
    __shared__ double sh[NR * 16];
    // the segment pass of this iteration has ended: its work counter starts
    // the next one from zero
    if (blockIdx.x == 0 && threadIdx.x == 0) *b.counter = 0u;
    const BChunk f = b.fold[blockIdx.x];   // blockIdx-indexed: scalar loads
    const BInst* I = b.inst + f.inst;
    if (!I->active) return;
    const int tid = threadIdx.x;
    const int jj = tid;
    const int64_t q = f.j0 + jj;   // library id
    const long long cnt1 = I->st[current(I->st)].cnt + 1;
    double x[NR];
    clear(x);
    if (q < I->n) {
        const int64_t j = I->pinv ? I->pinv[q] : q;   // caller product
        const unsigned long long tot = I->S_fx[q];
        I->S_fx[q] = 0ull;
        const double sj = (double)(long long)tot * I->inv_fx;
        I->S_d[j] = sj;
        x[R_P] = (double)((const T*)I->r)[j] * sj;
        const RowView rv{I->c, I->eta, I->tau_vec, I->tau_s, I->u_d, I->sum_u, 0};
        row_work<T>(rv, j, sj, cnt1, x);
    }
    block_reduce(x, sh);
    if (tid == 0) {
        double* p = b.bpart + (size_t)blockIdx.x * 8;
        for (int q = 0; q < NR; ++q) p[q] = x[q];
    }
}

template <typename T>
__global__ void __launch_bounds__(kRowThreads) k_bupdate(BArgs b)
{
    using namespace dual;
    __shared__ double sh[NR * 16];
    const BChunk rc = b.rows[blockIdx.x];
    const BInst* I = b.inst + rc.inst;
    if (!I->active) return;
    const int tid = threadIdx.x;
    double x[NR];
    clear(x);
    __shared__ long long zsh[kRowThreads / 64];
    const double Zd = fold_z(b.zpart, I->item0, I->item1, I->inv_z, zsh);
    // The partials of 64 products are combined four at a time in order, which
    // gives the single-instance fold's 256-product block partials bit for bit
    // (a block of 256 products adds its four waves' sums in that order); the
    // rest of the fold is the single instance's too, so both paths certify
    // the same gaps.
    const int nf = I->fold1 - I->fold0;
    for (int g = tid; g < (nf + 3) / 4; g += kRowThreads) {
        double y[NR];
        clear(y);
        for (int k = 0; k < 4; ++k) {
            const int q = 4 * g + k;
            double p[NR];
            clear(p);   // past the instance's last product: the values of empty waves
            if (q < nf)
                for (int r = 0; r < NR; ++r)
                    if (r != R_Z) p[r] = b.bpart[(size_t)(I->fold0 + q) * 8 + r];
            for (int r = 0; r < NR; ++r)
                y[r] = k == 0 ? p[r] : r == R_TH ? fmin(y[r], p[r]) : y[r] + p[r];
        }
        for (int r = 0; r < NR; ++r) x[r] = r == R_TH ? fmin(x[r], y[r]) : x[r] + y[r];
    }
    block_reduce(x, sh);
    x[R_Z] = Zd;   // the fixed-point sum, not the FP64 tree
    const double D = x[R_CETA] + x[R_Z];
    const int cur = current(I->st);
    DevState st = I->st[cur];
    double th = x[R_TH];
    const long long t1 = st.t + 1, cnt1 = st.cnt + 1;
    st.t = t1;
    if (D < st.dbest) st.dbest = D;
    st.sum_p += x[R_P];
    st.cnt = cnt1;
    if (t1 % b.check_every == 0) {
        const double cand = th * (st.sum_p / (double)cnt1);
        if (cand > st.lb) st.lb = cand;
    } else {
        th = 1.0;
    }
    double scale = 1.0;
    if (b.rule == SPFOM_STEP_POLYAK) {
        const double ex = D - st.lb;
        scale = (x[R_G] > 0.0 && ex > 0.0) ? b.gamma * ex / x[R_G] : 0.0;
    } else if (b.tau_decay > 0.0 && b.tau_decay < 1.0) {
        // the decaying constant step: tau_decay^k, k = (t - 1) / E, by
        // repeated FP64 products as the single-instance path forms it
        const long long k = (t1 - 1) / b.decay_every;
        for (long long q = 0; q < k; ++q) scale *= b.tau_decay;
    }
    st.scale = scale;
    bool restart = false;
    if (t1 == 1 || t1 == 2 * st.t0) {
        restart = true;
        st.t0 = t1;
        st.cnt = 0;
        st.sum_p = 0.0;
    }
    st.restart = restart ? 1 : 0;
    if (rc.j0 == 0 && tid == 0) {
        double* row = I->row;
        row[SPFOM_TR_DUAL] = D;
        row[SPFOM_TR_PRIMAL] = x[R_P];
        row[SPFOM_TR_Z] = x[R_Z];
        row[SPFOM_TR_ETA2] = x[R_E2];
        row[SPFOM_TR_INFEAS] = rel_infeas(x);
        row[SPFOM_TR_DBEST] = st.dbest;
        row[SPFOM_TR_LB] = st.lb;
        row[SPFOM_TR_GAP] = (st.dbest - st.lb) / fmax(fabs(st.dbest), DBL_MIN);
        row[SPFOM_TR_STEP] = scale;
        row[SPFOM_TR_THETA] = th;
        I->st[cur ^ 1] = st;
    }
    const int64_t i = rc.j0 + tid;
    if (i < I->m) {
        T* eta = (T*)I->eta;
        const T* tauv = (const T*)I->tau_vec;
        const double ti = scale * (tauv ? (double)tauv[i] : I->tau_s);
        double e = (double)eta[i];
        e = (1.0 - ti * b.mu) * e + ti * (I->u_d[i] - (double)((const T*)I->c)[i]);
        if (!(e > 0.0)) e = (e != e) ? e : 0.0;   // projection; NaN stays visible
        const T et = (T)e;
        eta[i] = et;
        if (restart) I->sum_u[i] = 0.0;
        ((T*)I->rho)[I->pnew ? I->pnew[i] : i] = ((const T*)I->r)[i] - et;
    }
}

// rho = r - eta for every instance (identity resource matrix)
template <typename T>
__global__ void __launch_bounds__(kRowThreads) k_bprices(const BInst* inst, const BChunk* rows)
{
    const BChunk rc = rows[blockIdx.x];
    const BInst* I = inst + rc.inst;
    const int64_t i = rc.j0 + threadIdx.x;
    if (i < I->n)
        ((T*)I->rho)[I->pnew ? I->pnew[i] : i] = ((const T*)I->r)[i] - ((const T*)I->eta)[i];
}

// Whole solves of small instances, one block each (a persistent launch): the
// block runs the iterations of its instance itself - the segment pass over its
// slot-major parts with the prices and every product's 64-bit bin in LDS, the
// fold in 64-product waves, the state update and the dual step - and tests the
// gap every check_every iterations as spfom_batch_solve does, so the batch
// needs one launch for the whole solve instead of three per iteration.  The
// products' state (c, eta, tau, r, the window sum of u, u) stays in LDS for the
// whole solve and goes back to the handle at the end.  The per-segment code,
// the integer sales and Z sums, the wave reductions and the four-at-a-time
// fold of the partials are those of k_bsegments, k_bfold and k_bupdate: the
// same bits.
constexpr int kSolveMaxProducts = 2048;   // products per instance of the one-launch form
struct BSolveArgs {
    int rule, check_every;
    double gamma, mu;
    double tau_decay;
    long long decay_every;
    long long max_iters;
    double tol;
    int* status;               // [count] CBLP_OK, CBLP_ENOTCONVERGED or CBLP_ENONFINITE
    long long* iters;          // [count] iterations run
};

// the LDS of one instance: bins [H], then per product (8-byte words) the
// prices, c, eta, tau, r, sum_u, u, then the fold partials [nf][8]
__host__ __device__ inline size_t bsolve_words(int H, int64_t n)
{
    return (size_t)H + 7 * (size_t)n + (size_t)((n + 63) / 64) * 8;
}

// NARROW: the instances may have pair and quad parts (FP32); without them
// only the 8-lane routine is compiled in, which keeps its registers.
template <typename T, typename IdxT, bool NARROW>
__global__ void __launch_bounds__(kSegThreads) k_bsolve(const BInst* __restrict__ inst, BSolveArgs sa)
{
    using namespace dual;
    extern __shared__ unsigned long long lds[];
    __shared__ double sh[NR * 16];
    __shared__ long long zsh[kSegThreads / 64];
    __shared__ DevState s_st;
    __shared__ double s_scale;
    __shared__ int s_restart, s_stop, s_status;
    const BInst* I = inst + blockIdx.x;
    if (!I->active) return;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int H = I->H;
    const int64_t n = I->n;   // = m (A = I)
    const int nf = (int)((n + 63) / 64);
    unsigned long long* bins = lds;
    T* lprice = (T*)(lds + H);                 // by library id
    double* c_l = (double*)(lds + H + n);      // the rest by caller product
    double* e_l = c_l + n;                     // eta, rounded to T as stored
    double* t_l = e_l + n;
    T* r_l = (T*)(t_l + n);
    double* su_l = (double*)(lds + H + 5 * n);
    double* u_l = su_l + n;
    double* part = u_l + n;
    const seg::FlatPrices<T> pr{(const T*)lprice};
    {
        const T* r = (const T*)I->r;
        const T* c = (const T*)I->c;
        const T* eta = (const T*)I->eta;
        const T* tauv = (const T*)I->tau_vec;
        for (int64_t j = tid; j < n; j += kSegThreads) {
            lprice[j] = ((const T*)I->rho)[j];
            c_l[j] = (double)c[j];
            e_l[j] = (double)eta[j];
            t_l[j] = tauv ? (double)tauv[j] : I->tau_s;
            r_l[j] = r[j];
            su_l[j] = I->sum_u[j];
            u_l[j] = 0.0;
        }
    }
    if (tid == 0) {
        s_st = I->st[current(I->st)];
        s_stop = 0;
        s_status = CBLP_ENOTCONVERGED;
    }
    for (long long it = 0; it < sa.max_iters; ++it) {
        for (int j = tid; j < H; j += kSegThreads) bins[j] = 0ull;
        __syncthreads();
        // the segment pass over the instance's parts
        ZAcc zacc;
        if constexpr (NARROW && sizeof(T) == 4) {
            const SegArgs& a0 = I->part_args[0];
            seg::process_tiles_pair<T, 8, seg::FlatPrices<T>, IdxT>(
                a0, 0, (a0.L + seg::kPairTileRows - 1) / seg::kPairTileRows, 1, bins, pr, zacc);
            const SegArgs& a1 = I->part_args[1];
            seg::process_tiles_quad<T, 8, seg::FlatPrices<T>, IdxT>(
                a1, 0, (a1.L + seg::kQuadTileRows - 1) / seg::kQuadTileRows, 1, bins, pr, zacc);
        }
        {
            const SegArgs& a2 = I->part_args[2];
            seg::process_tiles_slots<T, sizeof(T) == 4 ? 7 : 4, false, seg::FlatPrices<T>, IdxT>(
                a2, 0, (a2.L + kSegsPerTile - 1) / kSegsPerTile, 1, bins, pr, zacc);
        }
        __syncthreads();
        const long long zq = block_z(zacc, zsh);
        const double Zd = zq == kZPoison ? __longlong_as_double(0x7ff8000000000000ll)
                                         : (double)zq * I->inv_z;
        // the fold: 64 products (library ids) per wave, as k_bfold
        const long long cnt1 = s_st.cnt + 1;
        for (int f = wv; f < nf; f += kSegThreads / 64) {
            const int64_t q = (int64_t)f * 64 + lane;
            double x[NR];
            clear(x);
            if (q < n) {
                const int64_t j = I->pinv ? I->pinv[q] : q;   // caller product
                const double sj = (double)(long long)bins[q] * I->inv_fx;
                x[R_P] = (double)r_l[j] * sj;
                u_l[j] = sj;
                su_l[j] = row_work_values(c_l[j], e_l[j], t_l[j], su_l[j], sj, cnt1, 0, x);
            }
            wave_reduce(x);
            if (lane == 0)
                for (int q2 = 0; q2 < NR; ++q2) part[f * 8 + q2] = x[q2];
        }
        __syncthreads();
        // the partials four at a time, as k_bupdate, then the state
        double x[NR];
        clear(x);
        if (tid < kRowThreads)
            for (int g = tid; g < (nf + 3) / 4; g += kRowThreads) {
                double y[NR];
                clear(y);
                for (int k = 0; k < 4; ++k) {
                    const int q = 4 * g + k;
                    double p[NR];
                    clear(p);   // past the instance's last product: the values of empty waves
                    if (q < nf)
                        for (int rr = 0; rr < NR; ++rr)
                            if (rr != R_Z) p[rr] = part[q * 8 + rr];
                    for (int rr = 0; rr < NR; ++rr)
                        y[rr] = k == 0 ? p[rr] : rr == R_TH ? fmin(y[rr], p[rr]) : y[rr] + p[rr];
                }
                for (int rr = 0; rr < NR; ++rr) x[rr] = rr == R_TH ? fmin(x[rr], y[rr]) : x[rr] + y[rr];
            }
        block_reduce(x, sh, kRowThreads / 64);
        x[R_Z] = Zd;
        if (tid == 0) {
            const double D = x[R_CETA] + x[R_Z];
            DevState st = s_st;
            double th = x[R_TH];
            const long long t1 = st.t + 1;
            const long long c1 = st.cnt + 1;
            st.t = t1;
            if (D < st.dbest) st.dbest = D;
            st.sum_p += x[R_P];
            st.cnt = c1;
            if (t1 % sa.check_every == 0) {
                const double cand = th * (st.sum_p / (double)c1);
                if (cand > st.lb) st.lb = cand;
            } else {
                th = 1.0;
            }
            double scale = 1.0;
            if (sa.rule == SPFOM_STEP_POLYAK) {
                const double ex = D - st.lb;
                scale = (x[R_G] > 0.0 && ex > 0.0) ? sa.gamma * ex / x[R_G] : 0.0;
            } else if (sa.tau_decay > 0.0 && sa.tau_decay < 1.0) {
                const long long k = (t1 - 1) / sa.decay_every;
                for (long long q = 0; q < k; ++q) scale *= sa.tau_decay;
            }
            st.scale = scale;
            bool restart = false;
            if (t1 == 1 || t1 == 2 * st.t0) {
                restart = true;
                st.t0 = t1;
                st.cnt = 0;
                st.sum_p = 0.0;
            }
            st.restart = restart ? 1 : 0;
            s_st = st;
            s_scale = scale;
            s_restart = restart ? 1 : 0;
            // the trace row at the batch solve's tests: after every
            // check_every iterations and at the last one; a non-finite row
            // stops, a gap within tol converges
            if (t1 % sa.check_every == 0 || t1 == sa.max_iters) {
                double row[SPFOM_NTRACE];
                row[SPFOM_TR_DUAL] = D;
                row[SPFOM_TR_PRIMAL] = x[R_P];
                row[SPFOM_TR_Z] = x[R_Z];
                row[SPFOM_TR_ETA2] = x[R_E2];
                row[SPFOM_TR_INFEAS] = rel_infeas(x);
                row[SPFOM_TR_DBEST] = st.dbest;
                row[SPFOM_TR_LB] = st.lb;
                row[SPFOM_TR_GAP] = (st.dbest - st.lb) / fmax(fabs(st.dbest), DBL_MIN);
                row[SPFOM_TR_STEP] = scale;
                row[SPFOM_TR_THETA] = th;
                bool finite = true;
                for (int k = 0; k < SPFOM_NTRACE; ++k) {
                    I->row[k] = row[k];
                    finite = finite && isfinite(row[k]);
                }
                if (!finite) {
                    s_status = CBLP_ENONFINITE;
                    s_stop = 1;
                } else if (t1 % sa.check_every == 0 && row[SPFOM_TR_GAP] <= sa.tol) {
                    s_status = CBLP_OK;
                    s_stop = 1;
                }
            }
        }
        __syncthreads();
        // the dual step (eq. 16) of every row, and the prices for the next pass
        const double scale = s_scale;
        const bool restart = s_restart != 0;
        for (int64_t i = tid; i < n; i += kSegThreads) {
            const double ti = scale * t_l[i];
            double e = (1.0 - ti * sa.mu) * e_l[i] + ti * (u_l[i] - c_l[i]);
            if (!(e > 0.0)) e = (e != e) ? e : 0.0;   // projection; NaN stays visible
            const T et = (T)e;
            e_l[i] = (double)et;
            if (restart) su_l[i] = 0.0;
            lprice[I->pnew ? I->pnew[i] : i] = r_l[i] - et;
        }
        __syncthreads();
        if (s_stop) break;
    }
    // the instance's state back to the handle
    for (int64_t i = tid; i < n; i += kSegThreads) {
        const int64_t q = I->pnew ? I->pnew[i] : i;
        ((T*)I->eta)[i] = (T)e_l[i];
        ((T*)I->rho)[q] = lprice[q];
        I->sum_u[i] = su_l[i];
        I->u_d[i] = u_l[i];
        I->S_d[i] = u_l[i];
    }
    if (tid == 0) {
        DevState* st = (DevState*)I->st;
        st[0] = s_st;
        st[1] = s_st;
        sa.status[blockIdx.x] = s_status;
        sa.iters[blockIdx.x] = s_st.t;
    }
}

// Batched variants (the autotuner's candidates):
//   0  the row-major copies, prices gathered from global memory, no
//      cross-tile prefetch (no register spills)
//   1  the row-major copies, the item's instance prices copied into LDS,
//      ordered one-tile pipeline
//   2  the handles' own slot-major copies part by part, each part by the
//      groups of its width (2, 4 or 8 lanes), prices in LDS, 16-bit ids
//   3  the same over copies with 32-bit ids
constexpr int kBatchVariants = 4;
inline bool bseg_lds_prices(int variant) { return variant >= 1; }

template <typename T>
const void* bseg_fn(int variant)
{
    switch (variant) {
    case 1: return (const void*)k_bsegments<T, sizeof(T) == 4 ? 7 : 4, 3, 1>;
    case 2: return (const void*)k_bsegments<T, sizeof(T) == 4 ? 7 : 4, 3, 3, uint16_t>;
    case 3: return (const void*)k_bsegments<T, sizeof(T) == 4 ? 7 : 4, 3, 3, int32_t>;
    default: return (const void*)k_bsegments<T, 8, 0, 0>;
    }
}

int bfail(int code, const std::string& msg) { return set_error(code, msg); }

#define BHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return bfail(CBLP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace
}  // namespace cblp

using namespace cblp;

struct cblp_batch {
    int count = 0;
    int dtype = CBLP_F32;
    std::vector<cblp_instance*> hs;
    std::vector<BInst> h_inst;
    BInst* d_inst = nullptr;
    BItem* d_items = nullptr;
    int nitems = 0;
    int ipb = 4;                     // work items per segment block (the tuner may change it)
    size_t items_cap = 0, zpart_cap = 0;   // allocated entries
    std::vector<int> order;          // instances, largest first
    BChunk* d_fold = nullptr;
    int nfold = 0;
    BChunk* d_rows = nullptr;
    int nrows = 0;
    long long* zpart = nullptr;
    double* bpart = nullptr;
    DevState* st = nullptr;
    double* rows = nullptr;
    unsigned* counter = nullptr;
    double* pinned = nullptr;
    int grid = 1;
    int variant = 0;
    int Hmax = 1;
    int64_t nmax = 1;               // most products of any instance
    bool parts16_ok = false;        // every handle has a slot-major copy (any parts), 16-bit ids
    bool parts32_ok = false;        // the same with 32-bit ids
    hipStream_t stream = nullptr;    // the batch's own stream (graph capture needs one)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_K = 0;
    spfom_params graph_p{};          // the step parameters the graph was captured with
    std::vector<int64_t> t;          // per-instance iteration counts
    std::vector<int> mask;           // 1: the instance takes part in iterate and solve calls
    int persist = -1;                // whole solves in one launch: -1 small batches, 0 never, 1 always
    int* d_status = nullptr;         // [count] the persistent solve's outcome per instance
    long long* d_iters = nullptr;    // [count] its iterations
};

namespace {

// dynamic LDS of the batched segment kernel: the largest instance's bins, then
// (LDS-price variants) room for the largest instance's prices
size_t bseg_lds(const cblp_batch* b, int variant);
bool bseg_usable(const cblp_batch* b, int variant);


void batch_release(cblp_batch* b)
{
    if (!b) return;
    void* ptrs[] = {b->d_inst, b->d_items, b->d_fold, b->d_rows, b->zpart,
                    b->bpart, b->st, b->rows, b->counter, b->d_status, b->d_iters};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->pinned) (void)hipHostFree(b->pinned);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

template <typename P>
int balloc(P** p, size_t bytes)
{
    *p = nullptr;
    if (hipMalloc((void**)p, bytes ? bytes : 8) != hipSuccess) {
        (void)hipGetLastError();
        return bfail(CBLP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return CBLP_OK;
}

int check_bparams(const spfom_params* p)
{
    if (!p) return bfail(CBLP_EINVAL, "params is NULL");
    if (p->rule != SPFOM_STEP_CONST && p->rule != SPFOM_STEP_POLYAK)
        return bfail(CBLP_EINVAL, "unknown step rule");
    if (p->check_every < 1) return bfail(CBLP_EINVAL, "check_every must be >= 1");
    if (!(p->tau > 0.0 && std::isfinite(p->tau)) && !p->tau_vec)
        return bfail(CBLP_EINVAL, "tau must be finite and > 0");
    if (!(p->mu >= 0.0) || !std::isfinite(p->mu)) return bfail(CBLP_EINVAL, "mu must be >= 0");
    if (p->rule == SPFOM_STEP_POLYAK && !(p->gamma > 0.0 && p->gamma <= 2.0))
        return bfail(CBLP_EINVAL, "gamma must be in (0, 2]");
    if (p->bound != SPFOM_BOUND_GLOBAL)
        return bfail(CBLP_EINVAL, "batches certify with the global bound only");
    if (!(p->tau_decay >= 0.0 && p->tau_decay <= 1.0))
        return bfail(CBLP_EINVAL, "tau_decay must be in [0, 1]");
    if (p->tau_decay > 0.0 && p->tau_decay < 1.0 && p->decay_every < 1)
        return bfail(CBLP_EINVAL, "decay_every must be >= 1");
    return CBLP_OK;
}

// bind the callers' duals and steps into the instance table and upload it
int bind(cblp_batch* b, void* const* etas, const void* const* tau_vecs, const spfom_params* p,
         hipStream_t s)
{
    for (int q = 0; q < b->count; ++q) {
        if (!etas || !etas[q]) return bfail(CBLP_EINVAL, "NULL eta for instance " + std::to_string(q));
        b->h_inst[q].eta = etas[q];
        b->h_inst[q].tau_vec = tau_vecs ? tau_vecs[q] : nullptr;
        b->h_inst[q].tau_s = p->tau;
        if (!b->h_inst[q].tau_vec && !(p->tau > 0.0))
            return bfail(CBLP_EINVAL, "tau must be > 0 when an instance has no tau vector");
    }
    BHIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->count * sizeof(BInst),
                        hipMemcpyHostToDevice, s));
    return CBLP_OK;
}

int reset_states(cblp_batch* b, hipStream_t s)
{
    std::vector<DevState> st((size_t)b->count * 2);
    for (int q = 0; q < b->count; ++q) {
        std::memset(&st[2 * q], 0, 2 * sizeof(DevState));
        st[2 * q].dbest = st[2 * q + 1].dbest = INFINITY;
        st[2 * q + 1].t = -1;
    }
    BHIP(hipMemcpyAsync(b->st, st.data(), st.size() * sizeof(DevState), hipMemcpyHostToDevice, s));
    for (int q = 0; q < b->count; ++q)
        BHIP(hipMemsetAsync(b->hs[q]->sum_u, 0, (size_t)b->hs[q]->m * sizeof(double), s));
    BHIP(hipStreamSynchronize(s));
    std::fill(b->t.begin(), b->t.end(), 0);
    return CBLP_OK;
}

template <typename T>
int enqueue_iterations(cblp_batch* b, const spfom_params* p, int64_t iters, hipStream_t s)
{
    BArgs a;
    a.inst = b->d_inst;
    a.fold = b->d_fold;
    a.rows = b->d_rows;
    a.zpart = b->zpart;
    a.bpart = b->bpart;
    a.rule = p->rule;
    a.check_every = p->check_every;
    a.gamma = p->gamma;
    a.mu = p->mu;
    a.tau_decay = p->tau_decay;
    a.decay_every = p->decay_every;
    a.counter = b->counter;
    const size_t lds = bseg_lds(b, b->variant);
    const void* segf = bseg_fn<T>(b->variant);
    for (int64_t it = 0; it < iters; ++it) {
        void* sargs[] = {(void*)&b->d_inst, (void*)&b->d_items, (void*)&b->nitems,
                         (void*)&b->counter, (void*)&b->zpart,
                         (void*)&b->Hmax};
        BHIP(hipLaunchKernel(segf, dim3(b->grid), dim3(kSegThreads), sargs, lds, s));
        hipLaunchKernelGGL(k_bfold<T>, dim3(b->nfold), dim3(kFoldProducts), 0, s, a);
        hipLaunchKernelGGL(k_bupdate<T>, dim3(b->nrows), dim3(kRowThreads), 0, s, a);
        BHIP(hipGetLastError());
    }
    return CBLP_OK;
}

template <typename T>
int batch_prices(cblp_batch* b, hipStream_t s)
{
    hipLaunchKernelGGL(k_bprices<T>, dim3(b->nrows), dim3(kRowThreads), 0, s, b->d_inst, b->d_rows);
    BHIP(hipGetLastError());
    return CBLP_OK;
}

int run_iters(cblp_batch* b, const spfom_params* p, int64_t iters, hipStream_t s)
{
    return b->dtype == CBLP_F32 ? enqueue_iterations<float>(b, p, iters, s)
                                : enqueue_iterations<double>(b, p, iters, s);
}

int run_prices(cblp_batch* b, hipStream_t s)
{
    return b->dtype == CBLP_F32 ? batch_prices<float>(b, s) : batch_prices<double>(b, s);
}

// Whole solves in one launch (k_bsolve): every product of every instance has a
// 64-bit LDS bin, the handles have slot-major parts with one id type, and a
// block's bins, prices and fold partials fit its LDS.  Chosen by default when
// every instance has at most kSmallEntries entries: one block per instance
// then beats three launches per iteration.
constexpr int64_t kSmallEntries = 1 << 18;

size_t bsolve_lds(const cblp_batch* b) { return bsolve_words(b->Hmax, b->nmax) * 8; }

bool bsolve_ok(const cblp_batch* b)
{
    if (!(b->parts16_ok || b->parts32_ok)) return false;
    for (const cblp_instance* h : b->hs)
        if (h->n > h->Hb || h->n > kSolveMaxProducts) return false;
    int dev = 0, lmax = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return false;
    return bsolve_lds(b) + 2048 <= (size_t)lmax;
}

bool bsolve_small(const cblp_batch* b)
{
    for (const cblp_instance* h : b->hs)
        if (h->nnz > kSmallEntries) return false;
    return true;
}

template <typename T>
int launch_bsolve(cblp_batch* b, const spfom_params* p, hipStream_t s)
{
    if (!b->d_status) {
        if (hipMalloc((void**)&b->d_status, (size_t)b->count * sizeof(int)) != hipSuccess ||
            hipMalloc((void**)&b->d_iters, (size_t)b->count * sizeof(long long)) != hipSuccess) {
            (void)hipGetLastError();
            return bfail(CBLP_ENOMEM, "no memory for the persistent solve's outcome");
        }
    }
    BSolveArgs sa;
    sa.rule = p->rule;
    sa.check_every = p->check_every;
    sa.gamma = p->gamma;
    sa.mu = p->mu;
    sa.tau_decay = p->tau_decay;
    sa.decay_every = p->decay_every;
    sa.max_iters = p->max_iters;
    sa.tol = p->tol;
    sa.status = b->d_status;
    sa.iters = b->d_iters;
    bool narrow = false;   // some instance has rows for the 2- or 4-lane groups
    for (const cblp_instance* h : b->hs) narrow = narrow || h->quad_end > 0;
    const void* f = b->parts16_ok ? (narrow ? (const void*)k_bsolve<T, uint16_t, true>
                                            : (const void*)k_bsolve<T, uint16_t, false>)
                                  : (narrow ? (const void*)k_bsolve<T, int32_t, true>
                                            : (const void*)k_bsolve<T, int32_t, false>);
    const size_t lds = bsolve_lds(b);
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    void* args[] = {(void*)&b->d_inst, (void*)&sa};
    BHIP(hipLaunchKernel(f, dim3((unsigned)b->count), dim3(kSegThreads), args, lds, s));
    return CBLP_OK;
}

// join the batch stream to the caller's stream on entry and the other way on exit
int enter(cblp_batch* b, hipStream_t caller)
{
    BHIP(hipEventRecord(b->ev_in, caller));
    BHIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    return CBLP_OK;
}

int leave(cblp_batch* b, hipStream_t caller)
{
    BHIP(hipEventRecord(b->ev_out, b->stream));
    BHIP(hipStreamWaitEvent(caller, b->ev_out, 0));
    return CBLP_OK;
}

// capture check_every iterations once per K; replayed by spfom_batch_solve
size_t bseg_lds(const cblp_batch* b, int variant)
{
    const size_t esz = b->dtype == CBLP_F32 ? 4 : 8;
    return (size_t)b->Hmax * 8 + (bseg_lds_prices(variant) ? (size_t)b->nmax * esz : 0);
}

// a variant can run on this batch: its data exist and one block fits a CU
bool bseg_usable(const cblp_batch* b, int variant)
{
    if (variant < 0 || variant >= kBatchVariants) return false;
    if (variant == 2 && !b->parts16_ok) return false;
    if (variant == 3 && !b->parts32_ok) return false;
    const void* f = b->dtype == CBLP_F32 ? bseg_fn<float>(variant) : bseg_fn<double>(variant);
    const size_t lds = bseg_lds(b, variant);
    // a size past the device's LDS is refused here, not by the runtime (whose
    // error would stay behind as the thread's last error)
    int dev = 0, lmax = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        lds + 1024 > (size_t)lmax)
        return false;
    int per_cu = 0;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const bool ok = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kSegThreads, lds) ==
                        hipSuccess && per_cu >= 1;
    (void)hipGetLastError();
    return ok;
}

// The work list: each instance's parts cut into items of about equal tile
// count, ipb items per segment block on average, largest instance first;
// an item's length is a multiple of its part's block tile (512 positions in
// the pair layout, 256 in the quad layout, 128 in the 8-lane and row-major
// ones; parts start on multiples of 512), so that every item starts on a
// tile of its layout.  Sizes the Z partials, uploads the list and the
// instance table, and drops a captured graph (its launches hold the item
// count).
int build_items(cblp_batch* b, int ipb, hipStream_t s)
{
    int64_t total_tiles = 0;
    for (int q = 0; q < b->count; ++q) total_tiles += (b->hs[q]->L + kSegsPerTile - 1) / kSegsPerTile;
    const int64_t per_item = std::max<int64_t>(1, total_tiles / ((int64_t)b->grid * ipb));
    const int64_t align[3] = {seg::kPairTileRows, seg::kQuadTileRows, kSegsPerTile};
    std::vector<BItem> items;
    for (int q : b->order) {
        const cblp_instance* h = b->hs[q];
        BInst& I = b->h_inst[q];
        const int64_t pb[4] = {0, h->pair_end, h->quad_end, h->L};
        I.item0 = (int)items.size();
        for (int k = 0; k < 3; ++k) {
            const int64_t per_rows = (per_item * kSegsPerTile + align[k] - 1) / align[k] * align[k];
            for (int64_t p0 = pb[k]; p0 < pb[k + 1]; p0 += per_rows)
                items.push_back(BItem{q, k, p0, std::min(pb[k + 1], p0 + per_rows)});
        }
        I.item1 = (int)items.size();
    }
    auto grow = [&](void** ptr, size_t& cap, size_t need, size_t esz) -> int {
        need = std::max<size_t>(need, 1);
        if (need <= cap) return CBLP_OK;
        if (*ptr) (void)hipFree(*ptr);
        *ptr = nullptr;
        cap = 0;
        if (hipMalloc(ptr, need * esz) != hipSuccess) return bfail(CBLP_ENOMEM, "hipMalloc failed");
        cap = need;
        return CBLP_OK;
    };
    int rc;
    if ((rc = grow((void**)&b->d_items, b->items_cap, items.size(), sizeof(BItem))) ||
        (rc = grow((void**)&b->zpart, b->zpart_cap, items.size(), 8)))
        return rc;
    b->nitems = (int)items.size();
    b->ipb = ipb;
    if (!items.empty())
        BHIP(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(BItem),
                            hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->count * sizeof(BInst), hipMemcpyHostToDevice, s));
    BHIP(hipStreamSynchronize(s));
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
        b->graph_K = 0;
    }
    return CBLP_OK;
}

int ensure_graph(cblp_batch* b, const spfom_params* p)
{
    // the kernels' arguments hold the step rule's scalars: a graph serves only
    // the parameters it was captured with
    const spfom_params& g0 = b->graph_p;
    if (b->exec && b->graph_K == p->check_every && g0.rule == p->rule && g0.gamma == p->gamma &&
        g0.mu == p->mu && g0.tau_decay == p->tau_decay && g0.decay_every == p->decay_every)
        return CBLP_OK;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    hipGraph_t g = nullptr;
    BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = run_iters(b, p, p->check_every, b->stream);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return bfail(CBLP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return bfail(CBLP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    b->graph_K = p->check_every;
    b->graph_p = *p;
    return CBLP_OK;
}

}  // namespace

const std::vector<cblp_instance*>& cblp::batch_handles(cblp_batch_t b) { return b->hs; }

extern "C" {

int cblp_batch_create(cblp_batch_t* out, int32_t count, const cblp_t* handles, void* stream)
{
    set_error(CBLP_OK, "");
    if (!out || !handles || count < 1) return bfail(CBLP_EINVAL, "need out, handles and count >= 1");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    cblp_batch* b = new (std::nothrow) cblp_batch();
    if (!b) return bfail(CBLP_ENOMEM, "host allocation failed");
    auto bail = [&](int rc) {
        batch_release(b);
        return rc;
    };
    b->count = count;
    b->hs.assign(handles, handles + count);
    b->dtype = b->hs[0]->dtype;
    b->t.assign(count, 0);
    b->mask.assign(count, 1);
    int64_t Hmax = 1;
    for (int q = 0; q < count; ++q) {
        const cblp_instance* h = b->hs[q];
        if (!h) return bail(bfail(CBLP_EINVAL, "NULL handle " + std::to_string(q)));
        if (h->dtype != b->dtype) return bail(bfail(CBLP_EINVAL, "all instances need the same dtype"));
        if (h->a_ptr) return bail(bfail(CBLP_EINVAL, "batched solves need the identity resource matrix"));
        Hmax = std::max<int64_t>(Hmax, h->Hb);
    }
    b->Hmax = (int)Hmax;
    b->parts16_ok = true;
    b->parts32_ok = true;
    for (int q = 0; q < count; ++q) {
        b->nmax = std::max<int64_t>(b->nmax, b->hs[q]->n);
        // FP64 handles have one 8-lane part (the narrow groups are FP32 kernels)
        const bool parts = b->hs[q]->woff != nullptr &&
                           (b->dtype == CBLP_F32 || b->hs[q]->quad_end == 0);
        b->parts16_ok = b->parts16_ok && parts && b->hs[q]->idx16;
        b->parts32_ok = b->parts32_ok && parts && !b->hs[q]->idx16;
    }
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
        return bail(bfail(CBLP_EHIP, "stream or event creation failed"));

    // launch shape of the persistent segment kernel
    int cus = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->hs[0]->device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
    // default: the handles' slot-major copies with LDS prices when every
    // instance has them and they fit, else the spill-free global-price variant
    b->variant = bseg_usable(b, 2) ? 2 : bseg_usable(b, 3) ? 3 : bseg_usable(b, 1) ? 1 : 0;
    const size_t lds = bseg_lds(b, b->variant);
    int per_cu = 1;
    {
        const void* f = b->dtype == CBLP_F32 ? bseg_fn<float>(b->variant) : bseg_fn<double>(b->variant);
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kSegThreads, lds) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
    }
    b->grid = cus * per_cu;

    // instances largest first (the work list is built below, build_items)
    std::vector<int>& order = b->order;
    order.resize(count);
    for (int q = 0; q < count; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->hs[x]->nnz > b->hs[y]->nnz; });
    std::vector<BChunk> fold, rows;
    b->h_inst.assign(count, BInst());
    for (int q : order) {
        cblp_instance* h = b->hs[q];
        BInst& I = b->h_inst[q];
        std::memset(&I, 0, sizeof(I));
        SegArgs& a = I.seg;
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
        a.H = h->Hb;
        a.H64 = h->Hb;
        a.hp = 0;
        a.woff = h->woff;
        a.idx3 = h->idx3;
        a.v3 = h->v3;
        a.den3 = h->den3;
        a.S_fx = h->S_fx;
        a.fx_scale = h->fx_scale;
        a.zpart = nullptr;
        a.z_scale = h->z_scale;
        a.z_rmax = h->z_rmax;
        a.seg_R = nullptr;
        I.n = h->n;
        I.m = h->m;
        I.r = h->r;
        I.c = h->c;
        I.rho = h->rho;
        I.S_fx = h->S_fx;
        I.inv_fx = 1.0 / h->fx_scale;
        I.inv_z = 1.0 / h->z_scale;
        I.S_d = h->S_d;
        I.u_d = h->u_d;
        I.sum_u = h->sum_u;
        I.H = h->Hb;
        I.active = 1;
        I.pnew = h->pnew;
        I.pinv = h->pinv;
        // the parts of the slot-major copy: pair [0, P2), quad [P2, P4), 8-lane [P4, L)
        const int64_t P2 = h->pair_end, P4 = h->quad_end;
        const int64_t pb[4] = {0, P2, P4, h->L};
        const int64_t wo[3] = {0, h->woff_q, h->woff_b};
        for (int k = 0; k < 3; ++k) {
            SegArgs v = a;
            const size_t esz = h->esz;
            v.L = pb[k + 1] - pb[k];
            v.ptr = h->ptr2 + pb[k];
            v.vt0 = (const char*)h->vt0 + pb[k] * esz;
            v.lam = (const char*)h->lam2 + pb[k] * esz;
            v.Rwarm = (char*)h->Rwarm + pb[k] * esz;
            v.perm = h->perm + pb[k];
            v.woff = h->woff ? h->woff + wo[k] : nullptr;
            I.part_args[k] = v;
            I.pstart[k] = pb[k];
        }
        I.fold0 = (int)fold.size();
        for (int64_t j = 0; j < h->n; j += kFoldProducts) fold.push_back(BChunk{q, 0, j});
        I.fold1 = (int)fold.size();
        for (int64_t i = 0; i < h->m; i += kRowThreads) rows.push_back(BChunk{q, 0, i});
    }
    b->nfold = (int)fold.size();
    b->nrows = (int)rows.size();
    int rc;
    if ((rc = balloc(&b->d_inst, count * sizeof(BInst)))) return bail(rc);
    if ((rc = balloc(&b->d_fold, std::max<size_t>(fold.size(), 1) * sizeof(BChunk)))) return bail(rc);
    if ((rc = balloc(&b->d_rows, std::max<size_t>(rows.size(), 1) * sizeof(BChunk)))) return bail(rc);
    if ((rc = balloc(&b->bpart, std::max<size_t>(fold.size(), 1) * 8 * 8))) return bail(rc);
    if ((rc = balloc(&b->st, (size_t)count * 2 * sizeof(DevState)))) return bail(rc);
    if ((rc = balloc(&b->rows, (size_t)count * SPFOM_NTRACE * 8))) return bail(rc);
    if ((rc = balloc(&b->counter, 16))) return bail(rc);
    if (hipMemsetAsync(b->counter, 0, 16, s) != hipSuccess)   // then cleared by every k_bfold
        return bail(bfail(CBLP_EHIP, "hipMemsetAsync of the work counter failed"));
    if (hipHostMalloc((void**)&b->pinned, (size_t)count * SPFOM_NTRACE * 8, hipHostMallocDefault) != hipSuccess)
        return bail(bfail(CBLP_ENOMEM, "hipHostMalloc failed"));
    for (int q = 0; q < count; ++q) {
        b->h_inst[q].st = b->st + 2 * q;
        b->h_inst[q].row = b->rows + (size_t)q * SPFOM_NTRACE;
    }
    auto up = [&](void* d, const void* h, size_t n) {
        return n ? hipMemcpyAsync(d, h, n, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    if (up(b->d_fold, fold.data(), fold.size() * sizeof(BChunk)) != hipSuccess ||
        up(b->d_rows, rows.data(), rows.size() * sizeof(BChunk)) != hipSuccess ||
        hipMemsetAsync(b->rows, 0, (size_t)count * SPFOM_NTRACE * 8, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(bfail(CBLP_EHIP, "uploading the batch tables failed"));
    if ((rc = build_items(b, b->ipb, s))) return bail(rc);
    if ((rc = reset_states(b, s))) return bail(rc);
    *out = b;
    return CBLP_OK;
}

void cblp_batch_destroy(cblp_batch_t b) { batch_release(b); }

int spfom_batch_iterate(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                        const spfom_params* p, int64_t iters, double* rows_out, void* stream)
{
    set_error(CBLP_OK, "");
    if (!b) return bfail(CBLP_EINVAL, "batch is NULL");
    if (iters < 0) return bfail(CBLP_EINVAL, "iters < 0");
    int rc = check_bparams(p);
    if (rc) return rc;
    hipStream_t caller = (hipStream_t)stream;
    if ((rc = enter(b, caller))) return rc;
    for (int q = 0; q < b->count; ++q) b->h_inst[q].active = b->mask[q];
    if ((rc = bind(b, etas, tau_vecs, p, b->stream))) return rc;
    if ((rc = run_prices(b, b->stream))) return rc;
    if ((rc = run_iters(b, p, iters, b->stream))) return rc;
    for (int q = 0; q < b->count; ++q)
        if (b->h_inst[q].active) b->t[q] += iters;
    if (rows_out) {
        BHIP(hipMemcpyAsync(b->pinned, b->rows, (size_t)b->count * SPFOM_NTRACE * 8,
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipStreamSynchronize(b->stream));
        std::memcpy(rows_out, b->pinned, (size_t)b->count * SPFOM_NTRACE * 8);
    }
    return leave(b, caller);
}

int spfom_batch_solve(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                      const spfom_params* p, spfom_stats* outs, void* stream)
{
    set_error(CBLP_OK, "");
    if (!b || !outs) return bfail(CBLP_EINVAL, "NULL batch or outs");
    int rc = check_bparams(p);
    if (rc) return rc;
    if (p->max_iters < 0 || !(p->tol >= 0.0)) return bfail(CBLP_EINVAL, "need max_iters >= 0 and tol >= 0");
    hipStream_t caller = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = enter(b, caller))) return rc;
    for (int q = 0; q < b->count; ++q) b->h_inst[q].active = b->mask[q];
    if ((rc = bind(b, etas, tau_vecs, p, b->stream))) return rc;
    if ((rc = reset_states(b, b->stream))) return rc;
    if ((rc = ensure_graph(b, p))) return rc;
    if ((rc = run_prices(b, b->stream))) return rc;
    int live = 0;
    for (int q = 0; q < b->count; ++q) {
        std::memset(&outs[q], 0, sizeof(spfom_stats));
        outs[q].status = b->mask[q] ? CBLP_ENOTCONVERGED : CBLP_OK;
        live += b->mask[q];
    }
    const bool whole = live > 0 && p->max_iters > 0 && b->persist != 0 && bsolve_ok(b) &&
                       (b->persist == 1 || bsolve_small(b));
    if (whole) {   // every solve in one launch
        rc = b->dtype == CBLP_F32 ? launch_bsolve<float>(b, p, b->stream)
                                  : launch_bsolve<double>(b, p, b->stream);
        if (rc) return rc;
        std::vector<int> status((size_t)b->count);
        std::vector<long long> iters((size_t)b->count);
        BHIP(hipMemcpyAsync(status.data(), b->d_status, (size_t)b->count * sizeof(int),
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(iters.data(), b->d_iters, (size_t)b->count * sizeof(long long),
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipMemcpyAsync(b->pinned, b->rows, (size_t)b->count * SPFOM_NTRACE * 8,
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipStreamSynchronize(b->stream));
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (int q = 0; q < b->count; ++q) {
            if (!b->mask[q]) continue;
            spfom_stats& o = outs[q];
            o.iters = iters[q];
            b->t[q] = iters[q];
            std::memcpy(o.trace, b->pinned + (size_t)q * SPFOM_NTRACE, sizeof(o.trace));
            o.seconds = el;
            o.status = status[q];
        }
        live = 0;
    }
    // every active instance has done the same number of iterations t: run
    // blocks of K (the graph), the last one cut to max_iters - t (eager), and
    // test the gap after whole blocks only, as spfom_solve does
    const int64_t K = p->check_every;
    int64_t t = 0;
    while (live > 0 && t < p->max_iters) {
        const int64_t k = std::min<int64_t>(K, p->max_iters - t);
        if (k == K)
            BHIP(hipGraphLaunch(b->exec, b->stream));
        else if ((rc = run_iters(b, p, k, b->stream)))
            return rc;
        t += k;
        BHIP(hipMemcpyAsync(b->pinned, b->rows, (size_t)b->count * SPFOM_NTRACE * 8,
                            hipMemcpyDeviceToHost, b->stream));
        BHIP(hipStreamSynchronize(b->stream));
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        bool changed = false;
        for (int q = 0; q < b->count; ++q) {
            if (!b->h_inst[q].active) continue;
            b->t[q] += k;
            spfom_stats& o = outs[q];
            o.iters = b->t[q];
            std::memcpy(o.trace, b->pinned + (size_t)q * SPFOM_NTRACE, sizeof(o.trace));
            o.seconds = el;
            bool finite = true;
            for (int c = 0; c < SPFOM_NTRACE; ++c) finite = finite && std::isfinite(o.trace[c]);
            if (!finite) {
                o.status = CBLP_ENONFINITE;
            } else if (t % K == 0 && o.trace[SPFOM_TR_GAP] <= p->tol) {
                o.status = CBLP_OK;
            } else if (t < p->max_iters) {
                continue;
            }
            b->h_inst[q].active = 0;
            --live;
            changed = true;
        }
        if (changed && live > 0)
            BHIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->count * sizeof(BInst),
                                hipMemcpyHostToDevice, b->stream));
    }
    for (int q = 0; q < b->count; ++q) b->h_inst[q].active = b->mask[q];
    BHIP(hipMemcpyAsync(b->d_inst, b->h_inst.data(), b->count * sizeof(BInst),
                        hipMemcpyHostToDevice, b->stream));
    if ((rc = leave(b, caller))) return rc;
    for (int q = 0; q < b->count; ++q)
        if (outs[q].status != CBLP_OK)
            return bfail(outs[q].status, "instance " + std::to_string(q) + " did not reach tol");
    return CBLP_OK;
}

int cblp_batch_tune(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                    const spfom_params* p, int32_t iters, int32_t* chosen, void* stream)
{
    set_error(CBLP_OK, "");
    if (!b || iters < 1) return bfail(CBLP_EINVAL, "NULL batch or iters < 1");
    int rc = check_bparams(p);
    if (rc) return rc;
    hipStream_t caller = (hipStream_t)stream;
    if ((rc = enter(b, caller))) return rc;
    if ((rc = bind(b, etas, tau_vecs, p, b->stream))) return rc;
    if ((rc = run_prices(b, b->stream))) return rc;
    const int candidates[] = {0, 1, 2, 3};
    const int ipbs[] = {2, 4, 8, 16};   // work items per segment block
    double best = INFINITY;
    int best_v = b->variant, best_ipb = b->ipb;
    // the trial iterations move every handle's warm-start R*: keep a copy and
    // put it back, so that tuning leaves the handles as it found them
    std::vector<void*> saved(b->count, nullptr);
    for (int q = 0; q < b->count && !rc; ++q) {
        const cblp_instance* h = b->hs[q];
        const size_t bytes = (size_t)std::max<int64_t>(h->L, 1) * h->esz;
        if (hipMalloc(&saved[q], bytes) != hipSuccess) {
            saved[q] = nullptr;
            rc = bfail(CBLP_ENOMEM, "no memory for the warm starts");
        } else if (hipMemcpyAsync(saved[q], h->Rwarm, bytes, hipMemcpyDeviceToDevice, b->stream) !=
                   hipSuccess) {
            rc = bfail(CBLP_EHIP, "saving the warm starts failed");
        }
    }
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    const int keep = b->variant, keep_ipb = b->ipb;
    for (int ipb : ipbs) {
        if (rc) break;
        if ((rc = build_items(b, ipb, b->stream))) break;
        for (int v : candidates) {
            if (rc) break;
            if (!bseg_usable(b, v)) continue;
            b->variant = v;
            if ((rc = run_iters(b, p, 1, b->stream))) break;   // warm the variant
            BHIP(hipEventRecord(e0, b->stream));
            if ((rc = run_iters(b, p, iters, b->stream))) break;
            BHIP(hipEventRecord(e1, b->stream));
            BHIP(hipEventSynchronize(e1));
            float ms = 0.0f;
            BHIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_v = v;
                best_ipb = ipb;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int q = 0; q < b->count; ++q) {
        if (!saved[q]) continue;
        const cblp_instance* h = b->hs[q];
        const size_t bytes = (size_t)std::max<int64_t>(h->L, 1) * h->esz;
        if (hipMemcpyAsync(h->Rwarm, saved[q], bytes, hipMemcpyDeviceToDevice, b->stream) !=
                hipSuccess && !rc)
            rc = bfail(CBLP_EHIP, "restoring the warm starts failed");
    }
    (void)hipStreamSynchronize(b->stream);
    for (void* ptr : saved)
        if (ptr) (void)hipFree(ptr);
    b->variant = rc ? keep : best_v;
    const int rc_items = build_items(b, rc ? keep_ipb : best_ipb, b->stream);   // drops the graph
    if (!rc) rc = rc_items;
    if (chosen) *chosen = b->variant;
    if (!rc) rc = reset_states(b, b->stream);
    const int rc2 = leave(b, caller);
    return rc ? rc : rc2;
}

int cblp_batch_mask(cblp_batch_t b, const int32_t* take_part)
{
    set_error(CBLP_OK, "");
    if (!b) return bfail(CBLP_EINVAL, "batch is NULL");
    for (int q = 0; q < b->count; ++q) b->mask[q] = take_part ? (take_part[q] != 0) : 1;
    return CBLP_OK;
}

int cblp_batch_persistent(cblp_batch_t b, int32_t mode)
{
    set_error(CBLP_OK, "");
    if (!b) return bfail(CBLP_EINVAL, "NULL batch");
    if (mode < -1 || mode > 1) return bfail(CBLP_EINVAL, "mode must be -1, 0 or 1");
    if (mode == 1 && !bsolve_ok(b))
        return bfail(CBLP_EINVAL, "whole solves in one launch need every product in a 64-bit LDS bin "
                                  "and the handles' slot-major parts");
    b->persist = mode;
    return CBLP_OK;
}

int cblp_batch_select(cblp_batch_t b, int32_t variant)
{
    set_error(CBLP_OK, "");
    if (!b) return bfail(CBLP_EINVAL, "NULL batch");
    if (!bseg_usable(b, variant))
        return bfail(CBLP_EINVAL, "batch variant " + std::to_string(variant) + " cannot run on this batch");
    if (variant != b->variant && b->exec) {
        (void)hipGraphExecDestroy(b->exec);   // the captured graph holds the old kernel
        b->exec = nullptr;
    }
    b->variant = variant;
    return CBLP_OK;
}

int cblp_batch_info(cblp_batch_t b, int32_t* items, int32_t* grid, int32_t* variant)
{
    set_error(CBLP_OK, "");
    if (!b) return bfail(CBLP_EINVAL, "batch is NULL");
    if (items) *items = b->nitems;
    if (grid) *grid = b->grid;
    if (variant) *variant = b->variant;
    return CBLP_OK;
}

int cblp_batch_tune_cached(cblp_batch_t b, void* const* etas, const void* const* tau_vecs,
                           const spfom_params* p, int32_t iters, const char* cache_path,
                           int32_t* chosen, int32_t* items_per_block, void* stream)
{
    set_error(CBLP_OK, "");
    if (!b || !cache_path) return bfail(CBLP_EINVAL, "NULL batch or cache path");
    // key: the device's architecture and the batch's shape bucket
    std::string arch = "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->hs[0]->device) == hipSuccess) arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    int64_t nnz = 0, L = 0, nmax = 0;
    for (const cblp_instance* h : b->hs) {
        nnz += h->nnz;
        L += h->L;
        nmax = std::max<int64_t>(nmax, h->n);
    }
    auto lg = [](int64_t x) { int e = 0; std::frexp((double)x + 1.0, &e); return e; };
    const std::string key = arch + ":" + (b->dtype == CBLP_F32 ? "f32" : "f64") + ":count" +
                            std::to_string(b->count) + ":nnz2^" + std::to_string(lg(nnz)) +
                            ":L2^" + std::to_string(lg(L)) + ":n2^" + std::to_string(lg(nmax)) +
                            ":parts" + std::to_string((b->parts16_ok ? 1 : 0) + (b->parts32_ok ? 2 : 0));
    {
        FILE* f = std::fopen(cache_path, "r");
        if (f) {
            char kbuf[512];
            int v = -1, ipb = 0;
            int found_v = -1, found_ipb = 0;
            while (std::fscanf(f, "%511s %d %d", kbuf, &v, &ipb) == 3)
                if (key == kbuf) {   // the last entry for the key wins
                    found_v = v;
                    found_ipb = ipb;
                }
            std::fclose(f);
            if (found_v >= 0 && found_ipb >= 1 && found_ipb <= 64 && bseg_usable(b, found_v)) {
                hipStream_t caller = (hipStream_t)stream;
                int rc = enter(b, caller);
                if (!rc && found_v != b->variant && b->exec) {
                    (void)hipGraphExecDestroy(b->exec);
                    b->exec = nullptr;
                }
                if (!rc) b->variant = found_v;
                if (!rc) rc = build_items(b, found_ipb, b->stream);
                const int rc2 = leave(b, caller);
                if (rc || rc2) return rc ? rc : rc2;
                if (chosen) *chosen = b->variant;
                if (items_per_block) *items_per_block = b->ipb;
                return CBLP_OK;
            }
        }
    }
    int32_t v = 0;
    int rc = cblp_batch_tune(b, etas, tau_vecs, p, iters, &v, stream);
    if (rc) return rc;
    if (chosen) *chosen = v;
    if (items_per_block) *items_per_block = b->ipb;
    FILE* f = std::fopen(cache_path, "a");
    if (!f) return bfail(CBLP_EINVAL, std::string("cannot append to the tuning cache ") + cache_path);
    std::fprintf(f, "%s %d %d\n", key.c_str(), b->variant, b->ipb);
    std::fclose(f);
    return CBLP_OK;
}

}  // extern "C"

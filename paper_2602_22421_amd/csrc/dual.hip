// Dual phase of one iteration: sales totals, FP64 reductions, certified
// bound and the projected dual step (eq. 16).
//
//   k_fold_rows  (when a segment pass left rows of bins) S_j of the products
//             with LDS bins: the 64-bit sum over the pass's block rows
//   k_fold_lite  per product: S_j = (global 64-bit accumulator) / 2^bits and
//             P = sum r_j S_j; with A = I also the per-row work below
//   k_rows    (general A) per resource: u_i = sum_j a_ij S_j through A^T
//   per row   g_i = u_i - c_i; c.eta, sum (g)^+, the Polyak norm
//             sum tau_i g_i^2 (g zeroed where the projection binds), ||eta||^2
//             and the window sums of u for the certified bound
//   k_fold_step  (A = I, constant step) the rows' fold, the per-product
//             work and the dual step in one launch; the last block does
//             k_update's state work
//   k_update  every block folds the partials in the same fixed order, so all
//             blocks agree on D = c.eta + sum lambda R*, Dbest, the bound
//             LB = max over checks of theta * Pbar (theta = min_i min(1,
//             c_i / ubar_i)), the step multiplier and the window restart;
//             block 0 writes the next solver state and the trace row, every
//             block updates its rows: eta_i <- max(0, (1 - t_i mu) eta_i +
//             t_i g_i), rho_i = r_i - eta_i for A = I.
//
// The state is double-buffered (read st[t & 1], write st[(t + 1) & 1]), so
// no block waits for another and no device-wide fence is needed inside a
// kernel; kernel boundaries order the phases.  Every floating-point
// reduction has a fixed shape, so results are bitwise reproducible; sales
// totals are exact integer sums.
#include "dual_core.hpp"

namespace cblp {
namespace {

using namespace dual;

// Sums over products run in the library's order (products by falling
// popularity, library id q; caller product j = pinv[q]), where the sales sums
// and prices live; the arrays of the caller's products (r, c, eta, ...) are
// read and written at j.

// The segment blocks' rows into the sales sums: 64 products per block of 16
// waves, each wave adding every 16th row (one contiguous read per wave and
// row), the first wave the 16 partials.
__global__ void __launch_bounds__(64 * kStepWaves) k_fold_rows(PhaseArgs a)
{
    __shared__ unsigned long long part[kStepWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * 64 + lane;
    part[wv][lane] = row_bins_sum(a.brow, a.row_words, a.nrows, a.rows_H, a.rows_H64, q, wv,
                                  kStepWaves);
    __syncthreads();
    if (wv == 0 && q < a.rows_H) {
        unsigned long long t = 0ull;
#pragma unroll
        for (int w = 0; w < kStepWaves; ++w) t += part[w][lane];
        a.S_fx[q] += t;
    }
}

// Fold: one product per thread, kFoldLite threads per block.
template <typename T, bool IDENT>
__global__ void __launch_bounds__(kFoldLite) k_fold_lite(PhaseArgs a)
{
    __shared__ double sh[NR * 16];
    const int64_t q = (int64_t)blockIdx.x * kFoldLite + threadIdx.x;   // library id
    const long long cnt1 = a.mode == 0 ? a.st[a.par].cnt + 1 : 1;
    double x[NR];
    clear(x);
    if (q < a.n) {
        const int64_t j = a.pinv ? a.pinv[q] : q;   // caller product
        const unsigned long long tot = a.S_fx[q];
        if (!a.keep_sales) a.S_fx[q] = 0ull;
        const double sj = (double)(long long)tot * a.inv_fx;
        a.S_d[j] = sj;
        x[R_P] = (double)((const T*)a.r)[j] * sj;
        if (IDENT) row_work<T>(a, j, sj, cnt1, x);
    }
    block_reduce(x, sh);
    if (threadIdx.x == 0) store_part(a.bpart + (size_t)blockIdx.x * 8, x);
}

// A = I with a constant step while iterating: the step needs no global value
// (the multiplier is 1), so one launch does it all.  A block of 16 waves owns
// 64 products: the waves add the segment pass's rows for them, the first
// wave takes each product's sales, row work and dual step (eq. 16) and sums
// its values by the wave's shuffle tree; the last block to arrive (a
// counter; partials are published before it counts) folds the partials four
// at a time (the shape of k_fold_lite's 256-product blocks, so every path
// gives the same bits) into the solver state and the trace row.
template <typename T>
__global__ void __launch_bounds__(64 * kStepWaves) k_fold_step(PhaseArgs a)
{
    __shared__ double sh[NR * 16];
    __shared__ unsigned long long part[kStepWaves][64];
    __shared__ long long zsh[kStepWaves];
    __shared__ int s_last;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t q = (int64_t)blockIdx.x * 64 + lane;   // library id
    const bool own = wv == 0 && q < a.n;
    DevState st = a.st[a.par];
    const long long t1 = st.t + 1, cnt1 = st.cnt + 1;
    const bool restart = t1 == 1 || t1 == 2 * st.t0;   // averaging window restarts
    // the first wave's product values, loaded while the rows are read
    int64_t j = 0;
    unsigned long long tot = 0ull;
    double rj = 0.0, cj = 0.0, ej = 0.0, tj = 0.0, suj = 0.0;
    if (own) {
        j = a.pinv ? a.pinv[q] : q;   // caller product
        tot = a.S_fx[q];
        const T* tauv = (const T*)a.tau_vec;
        rj = (double)((const T*)a.r)[j];
        cj = (double)((const T*)a.c)[j];
        ej = (double)((const T*)a.eta)[j];
        tj = tauv ? (double)tauv[j] : a.tau_s;
        suj = a.sum_u[j];
    }
    part[wv][lane] = row_bins_sum(a.brow, a.row_words, a.nrows, a.rows_H, a.rows_H64, q, wv,
                                  kStepWaves);
    __syncthreads();
    if (wv == 0) {
        double x[NR];
        clear(x);
        if (own) {
#pragma unroll
            for (int w = 0; w < kStepWaves; ++w) tot += part[w][lane];
            a.S_fx[q] = 0ull;
            const double sj = (double)(long long)tot * a.inv_fx;
            a.S_d[j] = sj;
            x[R_P] = rj * sj;
            a.u_d[j] = sj;
            const double su = row_work_values(cj, ej, tj, suj, sj, cnt1, 0, x);
            const double ti = a.tau_mult * tj;
            double e = (1.0 - ti * a.mu) * ej + ti * (sj - cj);
            if (!(e > 0.0)) e = (e != e) ? e : 0.0;   // projection; NaN stays visible
            const T et = (T)e;
            ((T*)a.eta)[j] = et;
            a.sum_u[j] = restart ? 0.0 : su;
            ((T*)a.rho)[q] = ((const T*)a.r)[j] - et;
        }
        wave_reduce(x);
        if (lane == 0) {
            store_part(a.bpart + (size_t)blockIdx.x * 8, x);
            __threadfence();
            s_last = atomicAdd(a.arrive, 1u) == gridDim.x - 1 ? 1 : 0;
        }
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    double x[NR];
    const double Zd = fold_z(a.zpart, 0, a.nz, a.inv_z, zsh);
    fold_partials(a.bpart, (int)gridDim.x, x, sh);
    x[R_Z] = Zd;   // the fixed-point sum, not the FP64 tree
    if (tid != 0) return;
    const double D = x[R_CETA] + x[R_Z];
    double th = x[R_TH];
    st.t = t1;
    if (D < st.dbest) st.dbest = D;
    st.sum_p += x[R_P];
    st.cnt = cnt1;
    if (t1 % a.check_every == 0) {
        const double cand = th * (st.sum_p / (double)cnt1);
        if (cand > st.lb) st.lb = cand;
    } else {
        th = 1.0;
    }
    st.scale = a.tau_mult;
    if (restart) {
        st.t0 = t1;
        st.cnt = 0;
        st.sum_p = 0.0;
    }
    st.restart = restart ? 1 : 0;
    double* row = a.row;
    row[SPFOM_TR_DUAL] = D;
    row[SPFOM_TR_PRIMAL] = x[R_P];
    row[SPFOM_TR_Z] = x[R_Z];
    row[SPFOM_TR_ETA2] = x[R_E2];
    row[SPFOM_TR_INFEAS] = rel_infeas(x);
    row[SPFOM_TR_DBEST] = st.dbest;
    row[SPFOM_TR_LB] = st.lb;
    row[SPFOM_TR_GAP] = (st.dbest - st.lb) / fmax(fabs(st.dbest), DBL_MIN);
    row[SPFOM_TR_STEP] = a.tau_mult;
    row[SPFOM_TR_THETA] = th;
    a.st[a.par ^ 1] = st;
    *a.arrive = 0u;   // ready for the next launch
}

// u_i = sum_j a_ij S_j, one wave per resource row: lanes stride over the row's
// products, then a fixed shuffle tree (the result does not depend on timing)
__global__ void __launch_bounds__(256) k_rows_sum(PhaseArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= a.m) return;
    double u = 0.0;
    for (int64_t q = a.at_ptr[i] + lane; q < a.at_ptr[i + 1]; q += 64)
        u += a.at_val[q] * a.S_d[a.at_prod[q]];
    for (int o = 32; o > 0; o >>= 1) u += __shfl_down(u, o, 64);
    if (lane == 0) a.u_d[i] = u;
}

template <typename T>
__global__ void __launch_bounds__(kRowThreads) k_rows(PhaseArgs a)
{
    __shared__ double sh[NR * 16];
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + threadIdx.x;
    const long long cnt1 = a.mode == 0 ? a.st[a.par].cnt + 1 : 1;
    double x[NR];
    clear(x);
    if (i < a.m) row_work<T>(a, i, a.u_d[i], cnt1, x);
    block_reduce(x, sh);
    if (threadIdx.x == 0) store_part(a.bpart2 + (size_t)blockIdx.x * 8, x);
}

// Per-segment bound, step 1: theta of each product j (library id), the
// smallest c_i / ubar_i (at most 1) over the resources j uses; ubar is the
// window average including this iteration (row work has added u to sum_u).
template <typename T>
__global__ void __launch_bounds__(256) k_theta(PhaseArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n) return;
    const double cnt1 = (double)(a.st[a.par].cnt + 1);
    const T* c = (const T*)a.c;
    auto theta_i = [&](int64_t i) {
        const double ub = a.sum_u[i] / cnt1, ci = (double)c[i];
        return ub > ci ? ci / ub : 1.0;
    };
    double th = 1.0;
    if (!a.a_ptr) {
        th = theta_i(j);
    } else {
        for (int64_t q = a.a_ptr[j]; q < a.a_ptr[j + 1]; ++q) th = fmin(th, theta_i(a.a_idx[q]));
    }
    a.theta_prod[a.pnew ? a.pnew[j] : j] = th;
}

// Per-segment bound, step 2: sum over positions of theta_l pbar_l with
// theta_l the smallest theta of the products in N_l (1 for an empty set)
// and pbar_l = psum / (window length); one partial per block, fixed order.
__global__ void __launch_bounds__(256) k_pseg(PhaseArgs a)
{
    __shared__ double sh[4];
    const double cnt1 = (double)(a.st[a.par].cnt + 1);
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < a.L;
         p += (int64_t)gridDim.x * 256) {
        double tl = 1.0;
        for (int64_t q = a.ptr2[p]; q < a.ptr2[p + 1]; ++q) tl = fmin(tl, a.theta_prod[a.idx2[q]]);
        acc += tl * (a.psum[p] / cnt1);
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.pseg_part[blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

template <typename T, bool IDENT>
__global__ void __launch_bounds__(kRowThreads) k_update(PhaseArgs a)
{
    __shared__ double sh[NR * 16];
    const int tid = threadIdx.x;
    // every block folds all partials in the same order
    double x[NR];
    clear(x);
    __shared__ long long zsh[kRowThreads / 64];
    const double Zd = fold_z(a.zpart, 0, a.nz, a.inv_z, zsh);
    for (int q = tid; q < a.fold_blocks; q += kRowThreads) x[R_P] += a.bpart[(size_t)q * 8 + R_P];
    const double* rp = IDENT ? a.bpart : a.bpart2;
    const int nrow = IDENT ? a.fold_blocks : (int)gridDim.x;
    for (int q = tid; q < nrow; q += kRowThreads) {
        const double* p = rp + (size_t)q * 8;
        x[R_CETA] += p[R_CETA];
        x[R_INF] += p[R_INF];
        x[R_G] += p[R_G];
        x[R_TH] = fmin(x[R_TH], p[R_TH]);
        x[R_E2] += p[R_E2];
        x[R_CS] += p[R_CS];
    }
    block_reduce(x, sh);
    x[R_Z] = Zd;   // the fixed-point sum, not the FP64 tree
    const double D = x[R_CETA] + x[R_Z];
    const bool iter = a.mode != 1;      // a dual step follows
    const bool cert = a.mode == 0;      // full batch: dual bound and certificate
    double scale = 0.0;
    bool restart = false;
    DevState st = a.st[a.par];
    double th = x[R_TH];
    if (iter && !cert) {                // minibatch: the step only
        st.t += 1;
        scale = a.tau_mult;
        st.scale = scale;
    } else if (iter) {
        const long long t1 = st.t + 1, cnt1 = st.cnt + 1;
        st.t = t1;
        if (D < st.dbest) st.dbest = D;
        st.sum_p += x[R_P];
        st.cnt = cnt1;
        if (t1 % a.check_every == 0) {
            const double cand = th * (st.sum_p / (double)cnt1);
            if (cand > st.lb) st.lb = cand;
            if (a.pseg_part) {   // the per-segment bound, its partials in block order
                double ps = 0.0;
                for (int q = 0; q < a.pseg_blocks; ++q) ps += a.pseg_part[q];
                if (ps > st.lb) st.lb = ps;
            }
        } else {
            th = 1.0;
        }
        scale = a.tau_mult;
        if (a.rule == SPFOM_STEP_POLYAK) {
            const double ex = D - st.lb;
            scale = (x[R_G] > 0.0 && ex > 0.0) ? a.gamma * ex / x[R_G] : 0.0;
        }
        st.scale = scale;
        if (t1 == 1 || t1 == 2 * st.t0) {   // averaging window restarts
            restart = true;
            st.t0 = t1;
            st.cnt = 0;
            st.sum_p = 0.0;
        }
        st.restart = restart ? 1 : 0;
    }
    if (blockIdx.x == 0 && tid == 0) {
        double* row = a.row;
        row[SPFOM_TR_DUAL] = iter && !cert ? 0.0 : D;
        row[SPFOM_TR_PRIMAL] = x[R_P];
        row[SPFOM_TR_Z] = x[R_Z];
        row[SPFOM_TR_ETA2] = x[R_E2];
        row[SPFOM_TR_INFEAS] = rel_infeas(x);
        if (iter && !cert) {
            for (int q = SPFOM_TR_DBEST; q < SPFOM_NTRACE; ++q) row[q] = 0.0;
            row[SPFOM_TR_STEP] = scale;
            a.st[a.par ^ 1] = st;
        } else if (iter) {
            row[SPFOM_TR_DBEST] = st.dbest;
            row[SPFOM_TR_LB] = st.lb;
            row[SPFOM_TR_GAP] = (st.dbest - st.lb) / fmax(fabs(st.dbest), DBL_MIN);
            row[SPFOM_TR_STEP] = scale;
            row[SPFOM_TR_THETA] = th;
            a.st[a.par ^ 1] = st;
        } else {
            for (int q = SPFOM_TR_DBEST; q < SPFOM_NTRACE; ++q) row[q] = 0.0;
        }
    }
    if (!iter) return;
    const int64_t i = (int64_t)blockIdx.x * kRowThreads + tid;
    if (i < a.m) {
        T* eta = (T*)a.eta;
        const T* tauv = (const T*)a.tau_vec;
        const double ti = scale * (tauv ? (double)tauv[i] : a.tau_s);
        double e = (double)eta[i];
        e = (1.0 - ti * a.mu) * e + ti * (a.u_d[i] - (double)((const T*)a.c)[i]);
        if (!(e > 0.0)) e = (e != e) ? e : 0.0;   // projection; NaN stays visible
        const T et = (T)e;
        eta[i] = et;
        if (restart) a.sum_u[i] = 0.0;
        if (IDENT) ((T*)a.rho)[a.pnew ? a.pnew[i] : i] = ((const T*)a.r)[i] - et;
    }
}

template <typename T>
__global__ void k_prices_after(int64_t n, const T* r, const T* eta, const int64_t* a_ptr,
                               const int32_t* a_idx, const T* a_val, const int32_t* pnew,
                               T* rho)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    T x = r[j];
    for (int64_t q = a_ptr[j]; q < a_ptr[j + 1]; ++q) x -= a_val[q] * eta[a_idx[q]];
    rho[pnew ? pnew[j] : j] = x;
}

}  // namespace

template <typename T>
hipError_t launch_phase(const PhaseArgs& a, bool identity, hipStream_t s)
{
    const unsigned fold_grid = (unsigned)a.fold_blocks;
    const unsigned row_grid = (unsigned)((a.m + kRowThreads - 1) / kRowThreads);
    // per-segment bound at a check: theta per product, then per segment,
    // between the row work and the update (the two-kernel path)
    auto pseg = [&]() {
        if (!a.pseg_part) return;
        hipLaunchKernelGGL(k_theta<T>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_pseg, dim3((unsigned)a.pseg_blocks), dim3(256), 0, s, a);
    };
    if (identity && a.mode == 0 && a.rule != SPFOM_STEP_POLYAK && a.arrive && !a.pseg_part) {
        hipLaunchKernelGGL((k_fold_step<T>), dim3((unsigned)((a.n + 63) / 64)),
                           dim3(64 * kStepWaves), 0, s, a);
        return hipGetLastError();
    }
    if (a.nrows > 0 && a.rows_H > 0)
        hipLaunchKernelGGL(k_fold_rows, dim3((unsigned)((a.rows_H + 63) / 64)),
                           dim3(64 * kStepWaves), 0, s, a);
    if (identity) {
        hipLaunchKernelGGL((k_fold_lite<T, true>), dim3(fold_grid), dim3(kFoldLite), 0, s, a);
        pseg();
        hipLaunchKernelGGL((k_update<T, true>), dim3(row_grid), dim3(kRowThreads), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_fold_lite<T, false>), dim3(fold_grid), dim3(kFoldLite), 0, s, a);
        hipLaunchKernelGGL(k_rows_sum, dim3((unsigned)((a.m + 3) / 4)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_rows<T>, dim3(row_grid), dim3(kRowThreads), 0, s, a);
        pseg();
        hipLaunchKernelGGL((k_update<T, false>), dim3(row_grid), dim3(kRowThreads), 0, s, a);
        if (a.mode != 1) {   // a step was taken: rho = r - A^T eta
            const unsigned pg = (unsigned)((a.n + 255) / 256);
            hipLaunchKernelGGL(k_prices_after<T>, dim3(pg), dim3(256), 0, s, a.n,
                               (const T*)a.r, (const T*)a.eta, a.a_ptr, a.a_idx,
                               (const T*)a.a_val, a.pnew, (T*)a.rho);
        }
    }
    return hipGetLastError();
}

template hipError_t launch_phase<float>(const PhaseArgs&, bool, hipStream_t);
template hipError_t launch_phase<double>(const PhaseArgs&, bool, hipStream_t);

}  // namespace cblp

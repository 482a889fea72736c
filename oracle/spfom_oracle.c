/*
 * FP64 CPU oracle for full-batch SPFOM on the choice-based LP under the
 * generalized attraction model.  TEST INFRASTRUCTURE ONLY: the tests, the
 * package's smoke check and the benchmark's CPU-baseline leg may load it;
 * the solver library never does.  It shares no code with the HIP path.
 *
 * Plain, slow and written to be checked against the paper by eye:
 *
 *   Per-segment best response (the inner problem z_i of Section 4.1, in its
 *   GAM form).  The paper writes the sales-based LP for MNL (eqs. 5-9) and
 *   states that the CBLP/SBLP equivalence carries over to GAM (Section 3).
 *   Offering S to segment l gives choice probabilities
 *       pi_lj(S) = v_lj / (v_l0 + sum_{k in S} v_lk + sum_{k in N_l \ S} w_lk)
 *                = v_lj / (vt_l0 + sum_{k in S} vt_lk),
 *   with vt_l0 = v_l0 + sum_{k in N_l} w_lk and vt_lk = v_lk - w_lk > 0.
 *   The inner objective at reduced revenues rho_j = r_j - (A^T eta)_j is
 *   linear in the time shares x_l(S) of the CBLP (eqs. 1-4), so its maximum
 *   is lambda_l * R*_l with
 *       R(S) = sum_{j in S} rho_j v_lj / (vt_l0 + sum_{j in S} vt_lj),
 *       R*_l = max(0, max_S R(S))            (S = empty gives 0).
 *   A maximiser is a prefix of N_l sorted by key_lj = rho_j v_lj / vt_lj
 *   (the nested, prefix-closed family of Section 4.4); we take the
 *   shortest maximising prefix, i.e. S*_l = {j : key_lj > R*_l}, and sort
 *   ties by CSR position.  Sales s_lj = lambda_l v_lj / D_l on S*_l with
 *   D_l = vt_l0 + sum_{S*} vt_lj; z_l = lambda_l R*_l; p_l = sum r_j s_lj.
 *
 *   Iteration t (Algorithm 3 with every segment sampled):
 *       u^t = A S^t, S^t_j = sum_l s_lj
 *       eta^t_i = max(0, (1 - tau_i mu) eta^{t-1}_i - tau_i (c_i - u^t_i))   (eq. 16;
 *                 mu = 0 is the step of Algorithm 2)
 *   Dual bound  D^t = c . eta^{t-1} + sum_l z_l  (Lagrangian dual value of
 *   the minimax of Section 4.1, eqs. 10-14; >= OPT for any eta >= 0).
 *
 *   Step rules: CONST uses tau_i as given (the constant step of Algorithm 2,
 *   optionally one value per row; optionally shrunk by a factor tau_decay
 *   every decay_every iterations, a schedule of the build's own).  POLYAK scales the given tau_i by
 *   gamma (D^t - LB) / sum_i tau_i g_i^2 with g_i = u_i - c_i (zeroed where
 *   the projection is active); the paper fixes a constant step and stops on
 *   stagnation, this rule is the build's way to reach a certified tolerance.
 *
 *   Trace per iteration: D^t, P^t = sum_l p_l, Z^t = sum_l z_l, the squared
 *   norm of eta^{t-1} (the duals the pass was taken at, as D^t), the
 *   relative infeasibility ||(u^t - c)^+||_1 / ||c||_1 of the best
 *   responses, Dbest, LB, the gap, the step multiplier and theta.
 *
 *   Certified gap (the paper defines none): Dbest = min_t D^t >= OPT.  The
 *   primal average over the current window (window restarts at t = 1 and
 *   whenever t doubles the window start) has usage ubar and revenue Pbar;
 *   offering it a fraction theta = min(1, min_i c_i / ubar_i) of the time and
 *   the empty assortment otherwise is feasible, so LB = max over checks of
 *   theta * Pbar <= OPT.  With perseg, each segment l may instead be scaled
 *   by its own theta_l = min of c_i / ubar_i (and 1) over the resources i that
 *   a product of N_l uses: resource i then carries sum_l theta_l ubar_li <=
 *   (c_i / ubar_i) ubar_i = c_i, so sum_l theta_l pbar_l <= OPT as well (pbar_l
 *   the window average of p_l).  gap = (Dbest - LB) / |Dbest| (0 when both
 *   are 0).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NTRACE 10
/* trace columns */
enum { TR_D = 0, TR_P, TR_Z, TR_ETA2, TR_INFEAS, TR_DBEST, TR_LB, TR_GAP, TR_STEP, TR_THETA };

typedef struct {
    int64_t L, n, m;
    const int64_t* seg_ptr;
    const int32_t* idx;
    const double *v, *w, *v0, *lam, *r, *c;
    const int64_t* a_ptr;  /* NULL: A = identity (m == n) */
    const int32_t* a_idx;
    const double* a_val;
} orc_instance;

typedef struct {
    int32_t rule;          /* 0 CONST, 1 POLYAK */
    int32_t check_every;   /* K >= 1 */
    int32_t perseg;        /* 1: also the per-segment scaled bound */
    double gamma, mu;
    const double* tau;     /* [m] per-row step (CONST) or scaling (POLYAK) */
    double tau_decay;      /* CONST: step tau_i * tau_decay^k in iterations k*E+1..(k+1)*E */
    int64_t decay_every;   /* E (tau_decay 0 or 1: constant step) */
} orc_params;

/* The constant step's multiplier in iteration t (1-based): tau_decay^k with
 * k = (t - 1) / decay_every, multiplied out one factor at a time. */
static double orc_tau_mult(const orc_params* prm, int64_t t)
{
    if (prm->rule != 0 || !(prm->tau_decay > 0.0 && prm->tau_decay < 1.0)) return 1.0;
    double m = 1.0;
    for (int64_t q = 0; q < (t - 1) / prm->decay_every; ++q) m *= prm->tau_decay;
    return m;
}

typedef struct {
    int64_t t;             /* iterations done */
    int64_t t0;            /* window start */
    int64_t cnt;           /* iterations in window */
    double dbest, lb, sum_p;
    double* sum_u;         /* [m], owned by caller */
    double* sum_pl;        /* [L], owned by caller; used when perseg */
} orc_state;

typedef struct { double key; int64_t pos; } orc_item;

static int orc_cmp(const void* a, const void* b)
{
    const orc_item* x = (const orc_item*)a;
    const orc_item* y = (const orc_item*)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->pos < y->pos) ? -1 : (x->pos > y->pos);
}

/* Best response of one segment with k products.  rho, v, w are the segment's
 * entries in CSR order.  Writes R*, D_l and per-entry sales (0 off S*).
 * Returns |S*|, or -1 on allocation failure. */
int64_t orc_segment(int64_t k, const double* rho, const double* v, const double* w,
                    double v0, double lam, double* R_out, double* D_out,
                    double* s_out)
{
    double vt0 = v0;
    for (int64_t q = 0; q < k; ++q) vt0 += w[q];
    orc_item* it = (orc_item*)malloc((size_t)(k > 0 ? k : 1) * sizeof(orc_item));
    if (!it) return -1;
    for (int64_t q = 0; q < k; ++q) {
        it[q].key = rho[q] * v[q] / (v[q] - w[q]);
        it[q].pos = q;
    }
    qsort(it, (size_t)k, sizeof(orc_item), orc_cmp);
    /* prefix q = 0 is the empty assortment with R = 0 */
    double best = 0.0, num = 0.0, den = vt0, best_den = vt0;
    int64_t best_q = 0;
    for (int64_t q = 0; q < k; ++q) {
        int64_t p = it[q].pos;
        num += rho[p] * v[p];
        den += v[p] - w[p];
        double R = num / den;
        if (R > best) { best = R; best_q = q + 1; best_den = den; }
    }
    for (int64_t q = 0; q < k; ++q) s_out[q] = 0.0;
    for (int64_t q = 0; q < best_q; ++q) {
        int64_t p = it[q].pos;
        s_out[p] = lam * v[p] / best_den;
    }
    free(it);
    *R_out = best;
    *D_out = best_den;
    return best_q;
}

/* rho_j = r_j - sum_i a_ij eta_i */
static void orc_prices(const orc_instance* I, const double* eta, double* rho)
{
    for (int64_t j = 0; j < I->n; ++j) {
        double x = I->r[j];
        if (!I->a_ptr) {
            x -= eta[j];
        } else {
            for (int64_t q = I->a_ptr[j]; q < I->a_ptr[j + 1]; ++q)
                x -= I->a_val[q] * eta[I->a_idx[q]];
        }
        rho[j] = x;
    }
}

/* One best-response pass at fixed eta.  Outputs (each nullable except
 * Z, P): rho[n], S[n] product sales, u[m] resource usage, seg_R[L], seg_p[L],
 * sales[nnz].  Returns 0, or -1 on allocation failure. */
int orc_pass(const orc_instance* I, const double* eta, double* rho_out,
             double* S_out, double* u_out, double* seg_R, double* seg_p,
             double* sales_out, double* Z, double* P)
{
    int64_t kmax = 0;
    for (int64_t l = 0; l < I->L; ++l) {
        int64_t k = I->seg_ptr[l + 1] - I->seg_ptr[l];
        if (k > kmax) kmax = k;
    }
    double* rho = (double*)malloc((size_t)(I->n > 0 ? I->n : 1) * sizeof(double));
    double* S = (double*)calloc((size_t)(I->n > 0 ? I->n : 1), sizeof(double));
    double* buf = (double*)malloc((size_t)(kmax > 0 ? 4 * kmax : 4) * sizeof(double));
    if (!rho || !S || !buf) { free(rho); free(S); free(buf); return -1; }
    orc_prices(I, eta, rho);
    double z = 0.0, p = 0.0;
    double *rs = buf, *sv = buf + kmax;
    for (int64_t l = 0; l < I->L; ++l) {
        int64_t b = I->seg_ptr[l], k = I->seg_ptr[l + 1] - b;
        for (int64_t q = 0; q < k; ++q) rs[q] = rho[I->idx[b + q]];
        double R, D;
        if (orc_segment(k, rs, I->v + b, I->w + b, I->v0[l], I->lam[l], &R, &D, sv) < 0) {
            free(rho); free(S); free(buf); return -1;
        }
        double pl = 0.0;
        for (int64_t q = 0; q < k; ++q) {
            int32_t j = I->idx[b + q];
            S[j] += sv[q];
            pl += I->r[j] * sv[q];
            if (sales_out) sales_out[b + q] = sv[q];
        }
        z += I->lam[l] * R;
        p += pl;
        if (seg_R) seg_R[l] = R;
        if (seg_p) seg_p[l] = pl;
    }
    if (u_out) {
        if (!I->a_ptr) {
            memcpy(u_out, S, (size_t)I->m * sizeof(double));
        } else {
            for (int64_t i = 0; i < I->m; ++i) u_out[i] = 0.0;
            for (int64_t j = 0; j < I->n; ++j)
                for (int64_t q = I->a_ptr[j]; q < I->a_ptr[j + 1]; ++q)
                    u_out[I->a_idx[q]] += I->a_val[q] * S[j];
        }
    }
    if (rho_out) memcpy(rho_out, rho, (size_t)I->n * sizeof(double));
    if (S_out) memcpy(S_out, S, (size_t)I->n * sizeof(double));
    *Z = z;
    *P = p;
    free(rho); free(S); free(buf);
    return 0;
}

void orc_state_reset(orc_state* st, int64_t m)
{
    st->t = 0;
    st->t0 = 0;
    st->cnt = 0;
    st->dbest = INFINITY;
    st->lb = 0.0;
    st->sum_p = 0.0;
    for (int64_t i = 0; i < m; ++i) st->sum_u[i] = 0.0;
}

void orc_state_clear_segments(orc_state* st, int64_t L)
{
    for (int64_t l = 0; l < L; ++l) st->sum_pl[l] = 0.0;
}

/* Run `iters` iterations from eta (in/out), continuing the state st.
 * trace: nullable [iters x ORC_NTRACE].  Returns 0, -1 on allocation
 * failure. */
int orc_iterate(const orc_instance* I, const orc_params* prm, orc_state* st,
                int64_t iters, double* eta, double* trace)
{
    const int64_t m = I->m;
    double* u = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double* pl = (double*)malloc((size_t)(I->L > 0 ? I->L : 1) * sizeof(double));
    double* th = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    if (!u || !pl || !th) { free(u); free(pl); free(th); return -1; }
    for (int64_t it = 0; it < iters; ++it) {
        double Z, P;
        if (orc_pass(I, eta, NULL, NULL, u, NULL, pl, NULL, &Z, &P)) {
            free(u); free(pl); free(th); return -1;
        }
        st->t += 1;
        double ceta = 0.0;
        for (int64_t i = 0; i < m; ++i) ceta += I->c[i] * eta[i];
        double D = ceta + Z;
        if (D < st->dbest) st->dbest = D;
        for (int64_t i = 0; i < m; ++i) st->sum_u[i] += u[i];
        st->sum_p += P;
        if (prm->perseg)
            for (int64_t l = 0; l < I->L; ++l) st->sum_pl[l] += pl[l];
        st->cnt += 1;
        double theta = 1.0;
        if (st->t % prm->check_every == 0) {
            for (int64_t i = 0; i < m; ++i) {
                double ub = st->sum_u[i] / (double)st->cnt;
                th[i] = (ub > I->c[i]) ? I->c[i] / ub : 1.0;
                if (th[i] < theta) theta = th[i];
            }
            double cand = theta * (st->sum_p / (double)st->cnt);
            if (cand > st->lb) st->lb = cand;
            if (prm->perseg) {
                /* theta_l = min of theta_i over resources any product of N_l uses */
                double acc = 0.0;
                for (int64_t l = 0; l < I->L; ++l) {
                    double tl = 1.0;
                    for (int64_t q = I->seg_ptr[l]; q < I->seg_ptr[l + 1]; ++q) {
                        int32_t j = I->idx[q];
                        if (!I->a_ptr) {
                            if (th[j] < tl) tl = th[j];
                        } else {
                            for (int64_t e = I->a_ptr[j]; e < I->a_ptr[j + 1]; ++e)
                                if (th[I->a_idx[e]] < tl) tl = th[I->a_idx[e]];
                        }
                    }
                    acc += tl * (st->sum_pl[l] / (double)st->cnt);
                }
                if (acc > st->lb) st->lb = acc;
            }
        }
        /* step */
        double scale = orc_tau_mult(prm, st->t);
        if (prm->rule == 1) {
            double G = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                double g = u[i] - I->c[i];
                if (eta[i] <= 0.0 && g < 0.0) g = 0.0;
                G += prm->tau[i] * g * g;
            }
            double excess = D - st->lb;
            scale = (G > 0.0 && excess > 0.0) ? prm->gamma * excess / G : 0.0;
        }
        double infeas = 0.0, e2 = 0.0, csum = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            csum += I->c[i];
            double ti = scale * prm->tau[i];
            double g = u[i] - I->c[i];
            e2 += eta[i] * eta[i];          /* the duals the pass was taken at */
            double e = (1.0 - ti * prm->mu) * eta[i] + ti * g;
            eta[i] = e > 0.0 ? e : 0.0;
            if (g > 0.0) infeas += g;
        }
        if (trace) {
            double* tr = trace + it * ORC_NTRACE;
            tr[TR_D] = D;
            tr[TR_P] = P;
            tr[TR_Z] = Z;
            tr[TR_ETA2] = e2;
            tr[TR_INFEAS] = csum > 0.0 ? infeas / csum : infeas;   /* ||(u - c)^+||_1 / ||c||_1 */
            tr[TR_DBEST] = st->dbest;
            tr[TR_LB] = st->lb;
            tr[TR_GAP] = (st->dbest - st->lb) / fmax(fabs(st->dbest), DBL_MIN);
            tr[TR_STEP] = scale;
            tr[TR_THETA] = theta;
        }
        if (st->t == 1 || st->t == 2 * st->t0) {
            st->t0 = st->t;
            st->cnt = 0;
            st->sum_p = 0.0;
            for (int64_t i = 0; i < m; ++i) st->sum_u[i] = 0.0;
            if (prm->perseg)
                for (int64_t l = 0; l < I->L; ++l) st->sum_pl[l] = 0.0;
        }
    }
    free(u); free(pl); free(th);
    return 0;
}

/*
 * Stochastic minibatch SPFOM (Algorithm 2, Section 4.1; Algorithm 3 with
 * k B < L, Section 4.3).  The primal state is every segment's sales y_l
 * (y[nnz] in CSR order, caller-owned; y^0 as given, 0 for a cold start).
 * Iteration t takes the B distinct segments batch[t*B .. t*B+B-1] (drawn by
 * the caller), replaces their sales by the best response at eta^{t-1} and
 * leaves every other segment's sales as they were; the dual step then uses
 * the sales of ALL segments:
 *     S^t_j = sum_l y^t_lj,   u^t = A S^t,
 *     eta^t_i = max(0, (1 - tau_i mu) eta^{t-1}_i - tau_i (c_i - u^t_i)).
 * With B = L every segment is re-solved and this is orc_iterate's iteration.
 * Trace per iteration (other columns 0): P^t = sum_j r_j S^t_j, the squared
 * norm of eta^{t-1}, the relative infeasibility of u^t and the step
 * multiplier 1.  (No dual bound: that needs every segment's best response at
 * one eta; a full pass, orc_pass, gives it when wanted.)
 * Returns 0, or -1 on allocation failure.
 */
int orc_minibatch(const orc_instance* I, const orc_params* prm, int64_t iters, int64_t B,
                  const int32_t* batch, double* y, double* eta, double* trace)
{
    const int64_t m = I->m, n = I->n;
    int64_t kmax = 0;
    for (int64_t l = 0; l < I->L; ++l) {
        int64_t k = I->seg_ptr[l + 1] - I->seg_ptr[l];
        if (k > kmax) kmax = k;
    }
    double* rho = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double* S = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double* u = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    double* rs = (double*)malloc((size_t)(kmax > 0 ? kmax : 1) * sizeof(double));
    if (!rho || !S || !u || !rs) { free(rho); free(S); free(u); free(rs); return -1; }
    for (int64_t it = 0; it < iters; ++it) {
        orc_prices(I, eta, rho);
        /* re-solve the sampled segments at eta^{t-1} */
        for (int64_t q = 0; q < B; ++q) {
            const int64_t l = batch[it * B + q];
            const int64_t b = I->seg_ptr[l], k = I->seg_ptr[l + 1] - b;
            for (int64_t e = 0; e < k; ++e) rs[e] = rho[I->idx[b + e]];
            double R, D;
            if (orc_segment(k, rs, I->v + b, I->w + b, I->v0[l], I->lam[l], &R, &D, y + b) < 0) {
                free(rho); free(S); free(u); free(rs); return -1;
            }
        }
        /* the sales of every segment, sampled or not */
        for (int64_t j = 0; j < n; ++j) S[j] = 0.0;
        for (int64_t l = 0; l < I->L; ++l)
            for (int64_t e = I->seg_ptr[l]; e < I->seg_ptr[l + 1]; ++e) S[I->idx[e]] += y[e];
        if (!I->a_ptr) {
            memcpy(u, S, (size_t)m * sizeof(double));
        } else {
            for (int64_t i = 0; i < m; ++i) u[i] = 0.0;
            for (int64_t j = 0; j < n; ++j)
                for (int64_t e = I->a_ptr[j]; e < I->a_ptr[j + 1]; ++e)
                    u[I->a_idx[e]] += I->a_val[e] * S[j];
        }
        double P = 0.0;
        for (int64_t j = 0; j < n; ++j) P += I->r[j] * S[j];
        double infeas = 0.0, e2 = 0.0, csum = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const double ti = prm->tau[i];
            const double g = u[i] - I->c[i];
            csum += I->c[i];
            e2 += eta[i] * eta[i];
            const double e = (1.0 - ti * prm->mu) * eta[i] + ti * g;
            eta[i] = e > 0.0 ? e : 0.0;
            if (g > 0.0) infeas += g;
        }
        if (trace) {
            double* tr = trace + it * ORC_NTRACE;
            for (int c = 0; c < ORC_NTRACE; ++c) tr[c] = 0.0;
            tr[TR_P] = P;
            tr[TR_ETA2] = e2;
            tr[TR_INFEAS] = csum > 0.0 ? infeas / csum : infeas;
            tr[TR_STEP] = 1.0;
        }
    }
    free(rho); free(S); free(u); free(rs);
    return 0;
}

/*
 * SBLP -> CBLP recovery (Section 4.4, the recovery lemma), in the GAM form.
 * Given per-entry sales y[nnz] that satisfy the SBLP rows of each segment
 * (balance and scale), order each segment's products by y_lj / v_lj,
 * decreasing (ties by CSR position); S_l,q is the set of the first q
 * products.  Offering S with time share x(S) sells v_j / (vt_0 + sum_S vt)
 * per unit of time of each j in S, so nested sets reproduce y exactly when
 *     x(S_l,q) = (key_q - key_{q+1}) (vt_l0 + sum_{p<=q} vt_lp),
 * key_q = y / v of the q-th product (key_{k+1} = 0).  The probability of
 * offering S_l,q is alpha = x / lambda_l, and the empty set takes the rest.
 * (The lemma as printed leaves out the no-purchase term of the sum and
 * indexes the sets by [n]; both are read as above.)
 * Outputs: rank[e] = position of entry e in its segment's order (0-based),
 * alpha[e] = probability of the set of the entries ranked <= rank[e],
 * alpha0[l] = probability of the empty set.  lambda_l = 0 gives alpha = 0,
 * alpha0 = 1.  Returns 0, or -1 on allocation failure.
 */
int orc_recover(const orc_instance* I, const double* y, int32_t* rank, double* alpha,
                double* alpha0)
{
    int64_t kmax = 0;
    for (int64_t l = 0; l < I->L; ++l) {
        int64_t k = I->seg_ptr[l + 1] - I->seg_ptr[l];
        if (k > kmax) kmax = k;
    }
    orc_item* it = (orc_item*)malloc((size_t)(kmax > 0 ? kmax : 1) * sizeof(orc_item));
    if (!it) return -1;
    for (int64_t l = 0; l < I->L; ++l) {
        const int64_t b = I->seg_ptr[l], k = I->seg_ptr[l + 1] - b;
        double vt0 = I->v0[l];
        for (int64_t q = 0; q < k; ++q) vt0 += I->w[b + q];
        for (int64_t q = 0; q < k; ++q) {
            it[q].key = y[b + q] / I->v[b + q];
            it[q].pos = q;
        }
        qsort(it, (size_t)k, sizeof(orc_item), orc_cmp);
        double W = vt0, total = 0.0;
        for (int64_t q = 0; q < k; ++q) {
            const int64_t p = it[q].pos;
            W += I->v[b + p] - I->w[b + p];
            const double next = q + 1 < k ? it[q + 1].key : 0.0;
            const double x = (it[q].key - next) * W;
            const double a = I->lam[l] > 0.0 ? x / I->lam[l] : 0.0;
            rank[b + p] = (int32_t)q;
            alpha[b + p] = a;
            total += a;
        }
        alpha0[l] = I->lam[l] > 0.0 ? 1.0 - total : 1.0;
    }
    free(it);
    return 0;
}

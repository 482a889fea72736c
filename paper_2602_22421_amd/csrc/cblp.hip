// libcblp: full-batch SPFOM for the GAM choice-based LP on gfx950 (MI355X).
//
// One iteration (Algorithm 3 with every segment sampled, dual step eq. 16):
//   k_segments  per-segment exact best response (inner problem of Section 4.1,
//               GAM form) against reduced revenues rho = r - A^T eta, product
//               sales scattered into 64-bit fixed-point accumulators,
//               per-block FP64 partials of Z = sum_l lambda_l R*_l
//   k_dual      one workgroup: S -> u = A S, FP64 reductions (D, P, Z,
//               infeasibility, Polyak norm, certified bound), projected dual
//               step, next rho, trace row
//
// The per-segment solve.  With vt0 = v0 + sum_{N_l} w and vt_j = v_j - w_j,
// offering S earns revenue rate R(S) = sum_S rho_j v_j / (vt0 + sum_S vt_j)
// per arrival; R* = max(0, max_S R(S)) and S* = {j : rho_j v_j > R* vt_j}.
// R* is found by Dinkelbach's parametric iteration: starting at R = 0, take
// S(R) = {rho_j v_j > R vt_j} and set R <- R(S(R)) until S stops changing.
// The sequence increases and stops at R* after at most |N_l| + 1 rounds,
// usually 2-4; no sort and no division per product are needed.
//
// Layout: a 16-lane group (one DPP row) owns one segment; lane g holds
// products g, g+16, g+32, g+48 of the row in registers, products past 64 are
// re-read from memory in each round.  A 256-thread block holds 16 groups and
// strides over tiles of 16 consecutive segments, so the loads of one wave
// cover four neighbouring CSR rows.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "cblp.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(CBLP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kGroup = 16;            // lanes per segment
constexpr int kSegBlock = 256;        // threads per segment-kernel block
constexpr int kSegsPerTile = kSegBlock / kGroup;
constexpr int kJ = 4;                 // register-cached products per lane
constexpr int kDualBlock = 1024;

// ---------------------------------------------------------------- validation

enum : unsigned {
    V_IDX = 1u << 0, V_V = 1u << 1, V_W = 1u << 2, V_V0 = 1u << 3, V_LAM = 1u << 4,
    V_SEGPTR = 1u << 5, V_R = 1u << 6, V_C = 1u << 7, V_AIDX = 1u << 8, V_AVAL = 1u << 9,
    V_APTR = 1u << 10
};

const char* kValidationText[] = {
    "product index outside [0, n)", "attraction v not finite and > 0",
    "shadow attraction w outside [0, v)", "no-purchase attraction v0 not finite and > 0",
    "arrival rate lambda not finite and >= 0", "seg_ptr not non-decreasing from 0 to nnz",
    "revenue r not finite", "capacity c not finite and >= 0",
    "resource index outside [0, m)", "resource weight a not finite and >= 0",
    "a_ptr not non-decreasing from 0 to nnzA"};

template <typename T>
__global__ void k_validate(int64_t L, int64_t n, int64_t m, int64_t nnz, int64_t nnzA,
                           const int64_t* seg_ptr, const int32_t* idx, const T* v, const T* w,
                           const T* v0, const T* lam, const T* r, const T* c,
                           const int64_t* a_ptr, const int32_t* a_idx, const T* a_val,
                           unsigned* flags)
{
    unsigned bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t q = tid; q < nnz; q += stride) {
        int32_t j = idx[q];
        if (j < 0 || j >= n) bad |= V_IDX;
        T a = v[q], b = w[q];
        if (!(a > T(0)) || !isfinite(a)) bad |= V_V;
        if (!(b >= T(0)) || !(b < a)) bad |= V_W;
    }
    for (int64_t l = tid; l < L; l += stride) {
        T a = v0[l], b = lam[l];
        if (!(a > T(0)) || !isfinite(a)) bad |= V_V0;
        if (!(b >= T(0)) || !isfinite(b)) bad |= V_LAM;
        if (seg_ptr[l + 1] < seg_ptr[l]) bad |= V_SEGPTR;
    }
    if (tid == 0 && (seg_ptr[0] != 0 || seg_ptr[L] != nnz)) bad |= V_SEGPTR;
    for (int64_t j = tid; j < n; j += stride) {
        if (!isfinite(r[j])) bad |= V_R;
        if (a_ptr && a_ptr[j + 1] < a_ptr[j]) bad |= V_APTR;
    }
    for (int64_t i = tid; i < m; i += stride) {
        T x = c[i];
        if (!(x >= T(0)) || !isfinite(x)) bad |= V_C;
    }
    if (a_ptr) {
        if (tid == 0 && (a_ptr[0] != 0 || a_ptr[n] != nnzA)) bad |= V_APTR;
        for (int64_t q = tid; q < nnzA; q += stride) {
            int32_t i = a_idx[q];
            if (i < 0 || i >= m) bad |= V_AIDX;
            T x = a_val[q];
            if (!(x >= T(0)) || !isfinite(x)) bad |= V_AVAL;
        }
    }
    if (bad) atomicOr(flags, bad);
}

// vt0_l = v0_l + sum_{j in N_l} w_lj (FP64 sum, stored in T); block partial
// sums of lambda bound every product's sales for the fixed-point scale.
template <typename T>
__global__ void k_prepare(int64_t L, const int64_t* seg_ptr, const T* w, const T* v0,
                          const T* lam, T* vt0, double* lam_part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L;
         l += (int64_t)gridDim.x * blockDim.x) {
        double s = (double)v0[l];
        for (int64_t q = seg_ptr[l]; q < seg_ptr[l + 1]; ++q) s += (double)w[q];
        vt0[l] = (T)s;
        acc += (double)lam[l];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lam_part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------- prices

// rho_j = r_j - sum_i a_ij eta_i   (identity: r_j - eta_j)
template <typename T>
__global__ void k_prices(int64_t n, const T* r, const T* eta, const int64_t* a_ptr,
                         const int32_t* a_idx, const T* a_val, T* rho)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        T x = r[j];
        if (!a_ptr) {
            x -= eta[j];
        } else {
            for (int64_t q = a_ptr[j]; q < a_ptr[j + 1]; ++q) x -= a_val[q] * eta[a_idx[q]];
        }
        rho[j] = x;
    }
}

// ---------------------------------------------------------------- segments

template <typename X>
__device__ __forceinline__ X group_sum(X x)
{
    x += __shfl_xor(x, 8, kGroup);
    x += __shfl_xor(x, 4, kGroup);
    x += __shfl_xor(x, 2, kGroup);
    x += __shfl_xor(x, 1, kGroup);
    return x;
}

struct SegArgs {
    int64_t L;
    const int64_t* seg_ptr;
    const int32_t* idx;
    const void* v;
    const void* w;
    const void* vt0;
    const void* lam;
    const void* rho;
    unsigned long long* S_fx;   // [n] fixed-point product sales
    double fx_scale;            // 2^k
    double* part;               // [gridDim.x] FP64 partials of Z
    void* seg_R;                // [L] nullable
};

template <typename T>
__global__ void __launch_bounds__(kSegBlock) k_segments(SegArgs a)
{
    const T* __restrict__ v = (const T*)a.v;
    const T* __restrict__ w = (const T*)a.w;
    const T* __restrict__ rho = (const T*)a.rho;
    const int32_t* __restrict__ idx = a.idx;
    const int g = threadIdx.x & (kGroup - 1);
    const int grp = threadIdx.x / kGroup;
    double zacc = 0.0;

    const int64_t tiles = (a.L + kSegsPerTile - 1) / kSegsPerTile;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t l = tile * kSegsPerTile + grp;
        int64_t b = 0;
        int k = 0;
        T vt0 = T(1), lam = T(0);
        if (l < a.L) {
            b = a.seg_ptr[l];
            k = (int)(a.seg_ptr[l + 1] - b);
            vt0 = ((const T*)a.vt0)[l];
            lam = ((const T*)a.lam)[l];
        }
        // register cache: numerator term rho v, denominator term v - w
        T num[kJ], den[kJ], vv[kJ];
        int32_t id[kJ];
#pragma unroll
        for (int s = 0; s < kJ; ++s) {
            const int q = g + kGroup * s;
            if (q < k) {
                id[s] = idx[b + q];
                vv[s] = v[b + q];
                den[s] = vv[s] - w[b + q];
                num[s] = rho[id[s]] * vv[s];
            } else {
                id[s] = 0;
                vv[s] = T(0);
                den[s] = T(1);
                num[s] = T(0);   // never offered: 0 > R*1 fails for R >= 0
            }
        }
        auto sums = [&](T R, T& N, T& Dn, int& cnt) {
            T n_ = T(0), d_ = T(0);
            int c_ = 0;
#pragma unroll
            for (int s = 0; s < kJ; ++s) {
                if (num[s] > R * den[s]) {
                    n_ += num[s];
                    d_ += den[s];
                    ++c_;
                }
            }
            for (int q = kGroup * kJ + g; q < k; q += kGroup) {
                const T x = v[b + q];
                const T nn = rho[idx[b + q]] * x;
                const T dd = x - w[b + q];
                if (nn > R * dd) {
                    n_ += nn;
                    d_ += dd;
                    ++c_;
                }
            }
            N = group_sum(n_);
            Dn = group_sum(d_);
            cnt = group_sum(c_);
        };
        // Dinkelbach: R_cur defines the set whose sums are (N, Dn, cnt)
        T R = T(0), N, Dn;
        int cnt;
        sums(R, N, Dn, cnt);
        T Rstar = T(0);
        for (int round = 0; round < k + 2; ++round) {
            Rstar = cnt > 0 ? N / (vt0 + Dn) : T(0);
            T N2, D2;
            int c2;
            sums(Rstar, N2, D2, c2);
            if (c2 == cnt) break;
            R = Rstar;
            N = N2;
            Dn = D2;
            cnt = c2;
        }
        Rstar = cnt > 0 ? N / (vt0 + Dn) : T(0);
        // sales on S(R) = S(R*): s_j = lambda v_j / (vt0 + sum_S vt)
        const T Dl = vt0 + Dn;
#pragma unroll
        for (int s = 0; s < kJ; ++s) {
            if (num[s] > R * den[s]) {
                const T sj = lam * vv[s] / Dl;
                const long long q = __double2ll_rn((double)sj * a.fx_scale);
                atomicAdd(&a.S_fx[id[s]], (unsigned long long)q);
            }
        }
        for (int q = kGroup * kJ + g; q < k; q += kGroup) {
            const T x = v[b + q];
            const int32_t j = idx[b + q];
            if (rho[j] * x > R * (x - w[b + q])) {
                const T sj = lam * x / Dl;
                const long long qq = __double2ll_rn((double)sj * a.fx_scale);
                atomicAdd(&a.S_fx[j], (unsigned long long)qq);
            }
        }
        if (g == 0 && l < a.L) {
            zacc += (double)lam * (double)Rstar;
            if (a.seg_R) ((T*)a.seg_R)[l] = Rstar;
        }
    }
    __shared__ double sh[kSegBlock];
    sh[threadIdx.x] = zacc;
    __syncthreads();
    for (int o = kSegBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.part[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------- dual step

struct DevState {
    double dbest, lb, sum_p, pad;
    long long t, t0, cnt, pad2;
};

struct DualArgs {
    int64_t n, m;
    int nparts;
    int mode;                   // 0: iterate, 1: evaluate only
    int rule, check_every;
    double gamma, mu, tau_s;
    const void* tau_vec;        // [m] nullable
    const double* part;
    unsigned long long* S_fx;
    double inv_fx;
    const void* r;
    const void* c;
    void* eta;                  // [m] in/out (read-only in evaluate mode)
    void* rho;                  // [n] out
    const int64_t* a_ptr;       // CSC by product (NULL: identity)
    const int32_t* a_idx;
    const void* a_val;
    const int64_t* at_ptr;      // CSR by resource
    const int32_t* at_prod;
    const double* at_val;
    double* S_d;                // [n] scratch / output
    double* u_d;                // [m] scratch / output
    double* sum_u;              // [m] window sums
    DevState* st;
    double* row;                // trace row for this iteration
};

// Deterministic block reduction: a shuffle tree inside each wave, then every
// thread folds the wave results in wave order.
template <typename Op>
__device__ double block_reduce(double x, double* sh, Op op)
{
    for (int o = 32; o > 0; o >>= 1) x = op(x, __shfl_down(x, o, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (int)(blockDim.x >> 6);
    __syncthreads();
    if (lane == 0) sh[wave] = x;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < nw; ++q) r = op(r, sh[q]);
    return r;
}

struct AddOp {
    __device__ double operator()(double a, double b) const { return a + b; }
};
struct MinOp {
    __device__ double operator()(double a, double b) const { return a < b ? a : b; }
};

template <typename T, bool IDENT>
__global__ void __launch_bounds__(kDualBlock) k_dual(DualArgs a)
{
    __shared__ double sh[kDualBlock / 64];
    __shared__ double s_scale;
    __shared__ int s_restart;
    const int tid = threadIdx.x;
    const int BS = blockDim.x;
    const T* r = (const T*)a.r;
    const T* c = (const T*)a.c;
    T* eta = (T*)a.eta;
    const T* tauv = (const T*)a.tau_vec;
    const bool iter = a.mode == 0;

    const long long t1 = iter ? a.st->t + 1 : 0;
    const long long cnt1 = iter ? a.st->cnt + 1 : 1;

    double z = 0.0;
    for (int q = tid; q < a.nparts; q += BS) z += a.part[q];

    double P = 0.0;
    for (int64_t j = tid; j < a.n; j += BS) {
        const long long q = (long long)a.S_fx[j];
        a.S_fx[j] = 0ull;
        const double s = (double)q * a.inv_fx;
        a.S_d[j] = s;
        P += (double)r[j] * s;
    }
    if (!IDENT) __syncthreads();

    double ceta = 0.0, infeas = 0.0, G = 0.0, th = 1.0;
    for (int64_t i = tid; i < a.m; i += BS) {
        double u;
        if (IDENT) {
            u = a.S_d[i];
        } else {
            u = 0.0;
            for (int64_t q = a.at_ptr[i]; q < a.at_ptr[i + 1]; ++q)
                u += a.at_val[q] * a.S_d[a.at_prod[q]];
        }
        a.u_d[i] = u;
        const double ci = (double)c[i], ei = (double)eta[i];
        const double g = u - ci;
        ceta += ci * ei;
        if (g > 0.0) infeas += g;
        const double ti = tauv ? (double)tauv[i] : a.tau_s;
        const double gh = (ei <= 0.0 && g < 0.0) ? 0.0 : g;
        G += ti * gh * gh;
        if (iter) {
            const double su = a.sum_u[i] + u;
            a.sum_u[i] = su;
            const double ub = su / (double)cnt1;
            if (ub > ci) {
                const double x = ci / ub;
                if (x < th) th = x;
            }
        }
    }
    z = block_reduce(z, sh, AddOp());
    P = block_reduce(P, sh, AddOp());
    ceta = block_reduce(ceta, sh, AddOp());
    infeas = block_reduce(infeas, sh, AddOp());
    G = block_reduce(G, sh, AddOp());
    th = block_reduce(th, sh, MinOp());

    const double D = ceta + z;
    if (tid == 0) {
        double scale = 1.0;
        int restart = 0;
        if (iter) {
            DevState st = *a.st;
            st.t = t1;
            if (D < st.dbest) st.dbest = D;
            st.sum_p += P;
            st.cnt = cnt1;
            if (t1 % a.check_every == 0) {
                const double cand = th * (st.sum_p / (double)cnt1);
                if (cand > st.lb) st.lb = cand;
            } else {
                th = 1.0;
            }
            if (a.rule == SPFOM_STEP_POLYAK) {
                const double ex = D - st.lb;
                scale = (G > 0.0 && ex > 0.0) ? a.gamma * ex / G : 0.0;
            }
            a.row[SPFOM_TR_DBEST] = st.dbest;
            a.row[SPFOM_TR_LB] = st.lb;
            a.row[SPFOM_TR_GAP] = (st.dbest - st.lb) / fmax(fabs(st.dbest), DBL_MIN);
            a.row[SPFOM_TR_STEP] = scale;
            a.row[SPFOM_TR_THETA] = th;
            if (t1 == 1 || t1 == 2 * st.t0) {
                restart = 1;
                st.t0 = t1;
                st.cnt = 0;
                st.sum_p = 0.0;
            }
            *a.st = st;
        } else {
            for (int q = SPFOM_TR_DBEST; q < SPFOM_NTRACE; ++q) a.row[q] = 0.0;
        }
        a.row[SPFOM_TR_DUAL] = D;
        a.row[SPFOM_TR_PRIMAL] = P;
        a.row[SPFOM_TR_Z] = z;
        a.row[SPFOM_TR_INFEAS] = infeas;
        s_scale = scale;
        s_restart = restart;
    }
    __syncthreads();
    const double scale = s_scale;
    const int restart = s_restart;

    double e2 = 0.0;
    for (int64_t i = tid; i < a.m; i += BS) {
        double e = (double)eta[i];
        if (iter) {
            const double ti = scale * (tauv ? (double)tauv[i] : a.tau_s);
            e = (1.0 - ti * a.mu) * e + ti * (a.u_d[i] - (double)c[i]);
            if (!(e > 0.0)) e = e != e ? e : 0.0;   // keep NaN visible
            const T et = (T)e;
            eta[i] = et;
            e = (double)et;
            if (restart) a.sum_u[i] = 0.0;
        }
        e2 += e * e;
        if (IDENT) ((T*)a.rho)[i] = r[i] - (T)e;
    }
    if (!IDENT) {
        __syncthreads();
        const T* av = (const T*)a.a_val;
        for (int64_t j = tid; j < a.n; j += BS) {
            T x = r[j];
            for (int64_t q = a.a_ptr[j]; q < a.a_ptr[j + 1]; ++q) x -= av[q] * eta[a.a_idx[q]];
            ((T*)a.rho)[j] = x;
        }
    }
    e2 = block_reduce(e2, sh, AddOp());
    if (tid == 0) a.row[SPFOM_TR_ETA2] = e2;
}

}  // namespace

// ---------------------------------------------------------------- handle

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
    // owned
    void* vt0 = nullptr;
    void* rho = nullptr;
    unsigned long long* S_fx = nullptr;
    double* S_d = nullptr;
    double* u_d = nullptr;
    double* sum_u = nullptr;
    double* part = nullptr;
    DevState* st = nullptr;
    double* trace = nullptr;
    int64_t trace_rows = 0;
    int64_t* at_ptr = nullptr;
    int32_t* at_prod = nullptr;
    double* at_val = nullptr;
    double* pinned = nullptr;   // host staging for one trace row
    int seg_grid = 1;
    double fx_scale = 1.0;
    int64_t t = 0;              // host mirror of the iteration count
    // optional per-launch timing of the segment and dual kernels
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;   // (kernel id, index of start event)
};

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
    void* ptrs[] = {h->vt0, h->rho, h->S_fx, h->S_d, h->u_d, h->sum_u, h->part,
                    h->st, h->trace, h->at_ptr, h->at_prod, h->at_val};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->pinned) (void)hipHostFree(h->pinned);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

inline hipStream_t S(void* s) { return (hipStream_t)s; }

// Record an event pair around one kernel launch when timing is enabled.
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

int check_params(const cblp_instance* h, const spfom_params* p)
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
    (void)h;
    return CBLP_OK;
}

template <typename T>
int launch_prices(cblp_instance* h, const void* eta, hipStream_t s)
{
    const int blocks = (int)std::min<int64_t>((h->n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_prices<T>, dim3(std::max(blocks, 1)), dim3(256), 0, s, h->n,
                       (const T*)h->r, (const T*)eta, h->a_ptr, h->a_idx, (const T*)h->a_val,
                       (T*)h->rho);
    HIP_TRY(hipGetLastError());
    return CBLP_OK;
}

template <typename T>
int launch_segments(cblp_instance* h, void* seg_R, hipStream_t s)
{
    SegArgs a;
    a.L = h->L;
    a.seg_ptr = h->seg_ptr;
    a.idx = h->idx;
    a.v = h->v;
    a.w = h->w;
    a.vt0 = h->vt0;
    a.lam = h->lam;
    a.rho = h->rho;
    a.S_fx = h->S_fx;
    a.fx_scale = h->fx_scale;
    a.part = h->part;
    a.seg_R = seg_R;
    size_t slot;
    int rc = timed_begin(h, 0, s, &slot);
    if (rc) return rc;
    hipLaunchKernelGGL(k_segments<T>, dim3(h->seg_grid), dim3(kSegBlock), 0, s, a);
    HIP_TRY(hipGetLastError());
    return timed_end(h, slot, s);
}

template <typename T>
int launch_dual(cblp_instance* h, void* eta, const spfom_params* p, int mode, double* row,
                hipStream_t s)
{
    DualArgs a;
    a.n = h->n;
    a.m = h->m;
    a.nparts = h->seg_grid;
    a.mode = mode;
    a.rule = p ? p->rule : 0;
    a.check_every = p ? p->check_every : 1;
    a.gamma = p ? p->gamma : 1.0;
    a.mu = p ? p->mu : 0.0;
    a.tau_s = p ? p->tau : 1.0;
    a.tau_vec = p ? p->tau_vec : nullptr;
    a.part = h->part;
    a.S_fx = h->S_fx;
    a.inv_fx = 1.0 / h->fx_scale;
    a.r = h->r;
    a.c = h->c;
    a.eta = eta;
    a.rho = h->rho;
    a.a_ptr = h->a_ptr;
    a.a_idx = h->a_idx;
    a.a_val = h->a_val;
    a.at_ptr = h->at_ptr;
    a.at_prod = h->at_prod;
    a.at_val = h->at_val;
    a.S_d = h->S_d;
    a.u_d = h->u_d;
    a.sum_u = h->sum_u;
    a.st = h->st;
    a.row = row;
    size_t slot;
    int rc = timed_begin(h, 1, s, &slot);
    if (rc) return rc;
    if (h->a_ptr)
        hipLaunchKernelGGL((k_dual<T, false>), dim3(1), dim3(kDualBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_dual<T, true>), dim3(1), dim3(kDualBlock), 0, s, a);
    HIP_TRY(hipGetLastError());
    return timed_end(h, slot, s);
}

template <typename T>
int iterate_impl(cblp_instance* h, void* eta, const spfom_params* p, int64_t iters,
                 bool keep_trace, hipStream_t s)
{
    int rc = launch_prices<T>(h, eta, s);
    if (rc) return rc;
    for (int64_t it = 0; it < iters; ++it) {
        double* row = h->trace + (keep_trace ? it : 0) * SPFOM_NTRACE;
        if ((rc = launch_segments<T>(h, nullptr, s))) return rc;
        if ((rc = launch_dual<T>(h, eta, p, 0, row, s))) return rc;
        h->t += 1;
    }
    return CBLP_OK;
}

template <typename T>
int evaluate_impl(cblp_instance* h, const void* eta, void* seg_R, hipStream_t s)
{
    int rc = launch_prices<T>(h, eta, s);
    if (rc) return rc;
    if ((rc = launch_segments<T>(h, seg_R, s))) return rc;
    // evaluation leaves eta and the state untouched; rho is recomputed from
    // eta at the start of every iterate call
    return launch_dual<T>(h, const_cast<void*>(eta), nullptr, 1, h->trace, s);
}

int fill_stats(cblp_instance* h, spfom_stats* out, hipStream_t s, const double* dev_row)
{
    HIP_TRY(hipMemcpyAsync(h->pinned, dev_row, SPFOM_NTRACE * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (out) {
        out->iters = h->t;
        std::memcpy(out->trace, h->pinned, sizeof(out->trace));
        out->status = CBLP_OK;
        for (int q = 0; q < SPFOM_NTRACE; ++q)
            if (!std::isfinite(h->pinned[q])) out->status = CBLP_ENONFINITE;
    }
    for (int q = 0; q < SPFOM_NTRACE; ++q)
        if (!std::isfinite(h->pinned[q]))
            return fail(CBLP_ENONFINITE, "non-finite value in trace column " + std::to_string(q));
    return CBLP_OK;
}

int reset_state(cblp_instance* h, hipStream_t s)
{
    DevState st;
    std::memset(&st, 0, sizeof(st));
    st.dbest = INFINITY;
    HIP_TRY(hipMemcpyAsync(h->st, &st, sizeof(st), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(h->sum_u, 0, (size_t)std::max<int64_t>(h->m, 1) * sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    h->t = 0;
    return CBLP_OK;
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

const char* cblp_last_error(void) { return g_err.c_str(); }

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
    if (dtype != CBLP_F32 && dtype != CBLP_F64) return fail(CBLP_EINVAL, "dtype must be CBLP_F32 or CBLP_F64");
    if (!seg_ptr || !r || !c || (L > 0 && (!v0 || !lambda)))
        return fail(CBLP_EINVAL, "NULL instance array");
    const bool ident = !a_ptr && !a_idx && !a_val;
    if (!ident && (!a_ptr || !a_idx || !a_val))
        return fail(CBLP_EINVAL, "a_ptr, a_idx, a_val must be all NULL or all set");
    if (ident && m != n) return fail(CBLP_EINVAL, "identity resource matrix needs m == n");
    hipStream_t s = S(stream);

    cblp_instance* h = new (std::nothrow) cblp_instance();
    if (!h) return fail(CBLP_ENOMEM, "host allocation failed");
    auto bail = [&](int rc) { release(h); return rc; };
    if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(CBLP_EHIP, "hipGetDevice failed"));
    h->dtype = dtype;
    h->esz = dtype == CBLP_F32 ? 4 : 8;
    h->L = L; h->n = n; h->m = m;
    h->seg_ptr = seg_ptr; h->idx = prod_idx; h->v = v; h->w = w; h->v0 = v0; h->lam = lambda;
    h->r = r; h->c = c; h->a_ptr = a_ptr; h->a_idx = a_idx; h->a_val = a_val;

    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, seg_ptr + L, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return bail(fail(CBLP_EHIP, "reading seg_ptr[L] failed"));
    if (nnz < 0) return bail(fail(CBLP_EINVAL, "seg_ptr[L] < 0"));
    if (nnz > 0 && (!prod_idx || !v || !w)) return bail(fail(CBLP_EINVAL, "NULL CSR array"));
    h->nnz = nnz;
    std::vector<int64_t> hap;
    if (!ident) {
        hap.resize((size_t)n + 1);
        if (hipMemcpyAsync(hap.data(), a_ptr, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return bail(fail(CBLP_EHIP, "reading a_ptr failed"));
        h->nnzA = hap[n];
        if (h->nnzA < 0) return bail(fail(CBLP_EINVAL, "a_ptr[n] < 0"));
    }

    // validation
    unsigned* dflags = nullptr;
    int rc = dalloc(&dflags, sizeof(unsigned));
    if (rc) return bail(rc);
    unsigned flags = 0;
    {
        const int blocks = 1024;
        if (hipMemsetAsync(dflags, 0, sizeof(unsigned), s) != hipSuccess) {
            (void)hipFree(dflags);
            return bail(fail(CBLP_EHIP, "hipMemsetAsync failed"));
        }
        if (dtype == CBLP_F32)
            hipLaunchKernelGGL(k_validate<float>, dim3(blocks), dim3(256), 0, s, L, n, m, nnz,
                               h->nnzA, seg_ptr, prod_idx, (const float*)v, (const float*)w,
                               (const float*)v0, (const float*)lambda, (const float*)r,
                               (const float*)c, a_ptr, a_idx, (const float*)a_val, dflags);
        else
            hipLaunchKernelGGL(k_validate<double>, dim3(blocks), dim3(256), 0, s, L, n, m, nnz,
                               h->nnzA, seg_ptr, prod_idx, (const double*)v, (const double*)w,
                               (const double*)v0, (const double*)lambda, (const double*)r,
                               (const double*)c, a_ptr, a_idx, (const double*)a_val, dflags);
        hipError_t e1 = hipGetLastError();
        hipError_t e2 = hipMemcpyAsync(&flags, dflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
        hipError_t e3 = hipStreamSynchronize(s);
        (void)hipFree(dflags);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            return bail(fail(CBLP_EHIP, "validation kernel failed"));
    }
    if (flags) {
        std::string msg = "invalid instance:";
        for (int b = 0; b < 11; ++b)
            if (flags & (1u << b)) msg += std::string(" ") + kValidationText[b] + ";";
        return bail(fail(CBLP_EINVAL, msg));
    }

    // workspace
    const size_t esz = h->esz;
    if ((rc = dalloc(&h->vt0, (size_t)std::max<int64_t>(L, 1) * esz))) return bail(rc);
    if ((rc = dalloc(&h->rho, (size_t)n * esz))) return bail(rc);
    if ((rc = dalloc(&h->S_fx, (size_t)n * 8))) return bail(rc);
    if ((rc = dalloc(&h->S_d, (size_t)n * 8))) return bail(rc);
    if ((rc = dalloc(&h->u_d, (size_t)m * 8))) return bail(rc);
    if ((rc = dalloc(&h->sum_u, (size_t)m * 8))) return bail(rc);
    if ((rc = dalloc(&h->st, sizeof(DevState)))) return bail(rc);
    if ((rc = ensure_trace(h, 64))) return bail(rc);
    if (hipHostMalloc((void**)&h->pinned, SPFOM_NTRACE * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return bail(fail(CBLP_ENOMEM, "hipHostMalloc failed"));

    // segment-kernel grid: enough blocks to fill the chip, strided over tiles
    {
        int cus = 256;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) cus = prop.multiProcessorCount;
        const int64_t tiles = (L + kSegsPerTile - 1) / kSegsPerTile;
        h->seg_grid = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)cus * 8));
    }
    if ((rc = dalloc(&h->part, (size_t)h->seg_grid * sizeof(double)))) return bail(rc);

    // vt0 and the arrival-rate total that bounds every product's sales
    {
        const int pblocks = 256;
        double* lp = nullptr;
        if ((rc = dalloc(&lp, pblocks * sizeof(double)))) return bail(rc);
        if (dtype == CBLP_F32)
            hipLaunchKernelGGL(k_prepare<float>, dim3(pblocks), dim3(256), 0, s, L, seg_ptr,
                               (const float*)w, (const float*)v0, (const float*)lambda,
                               (float*)h->vt0, lp);
        else
            hipLaunchKernelGGL(k_prepare<double>, dim3(pblocks), dim3(256), 0, s, L, seg_ptr,
                               (const double*)w, (const double*)v0, (const double*)lambda,
                               (double*)h->vt0, lp);
        std::vector<double> hl(pblocks);
        hipError_t e1 = hipGetLastError();
        hipError_t e2 = hipMemcpyAsync(hl.data(), lp, pblocks * sizeof(double), hipMemcpyDeviceToHost, s);
        hipError_t e3 = hipStreamSynchronize(s);
        (void)hipFree(lp);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            return bail(fail(CBLP_EHIP, "prepare kernel failed"));
        double tot = 0.0;
        for (double x : hl) tot += x;
        // every product's sales are at most sum_l lambda_l; keep 2 bits of headroom
        int e = 0;
        std::frexp(tot + 1.0, &e);
        const int bits = std::min(60, 61 - e);
        if (bits < 8) return bail(fail(CBLP_EINVAL, "arrival rates too large for the 64-bit sales accumulator"));
        h->fx_scale = std::ldexp(1.0, bits);
    }

    // A^T (CSR by resource) for u = A S, built on the host once
    if (!ident) {
        const int64_t nA = h->nnzA;
        std::vector<int32_t> ai((size_t)std::max<int64_t>(nA, 1));
        std::vector<double> av((size_t)std::max<int64_t>(nA, 1));
        std::vector<float> avf;
        bool ok = true;
        if (nA > 0) {
            ok &= hipMemcpyAsync(ai.data(), a_idx, nA * sizeof(int32_t), hipMemcpyDeviceToHost, s) == hipSuccess;
            if (dtype == CBLP_F32) {
                avf.resize((size_t)nA);
                ok &= hipMemcpyAsync(avf.data(), a_val, nA * sizeof(float), hipMemcpyDeviceToHost, s) == hipSuccess;
            } else {
                ok &= hipMemcpyAsync(av.data(), a_val, nA * sizeof(double), hipMemcpyDeviceToHost, s) == hipSuccess;
            }
            ok &= hipStreamSynchronize(s) == hipSuccess;
        }
        if (!ok) return bail(fail(CBLP_EHIP, "reading the resource matrix failed"));
        if (dtype == CBLP_F32)
            for (int64_t q = 0; q < nA; ++q) av[q] = avf[q];
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
                tval[dst] = av[q];
            }
        if ((rc = dalloc(&h->at_ptr, (m + 1) * sizeof(int64_t)))) return bail(rc);
        if ((rc = dalloc(&h->at_prod, std::max<int64_t>(nA, 1) * sizeof(int32_t)))) return bail(rc);
        if ((rc = dalloc(&h->at_val, std::max<int64_t>(nA, 1) * sizeof(double)))) return bail(rc);
        ok = hipMemcpyAsync(h->at_ptr, tp.data(), (m + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s) == hipSuccess;
        if (nA > 0) {
            ok &= hipMemcpyAsync(h->at_prod, tprod.data(), nA * sizeof(int32_t), hipMemcpyHostToDevice, s) == hipSuccess;
            ok &= hipMemcpyAsync(h->at_val, tval.data(), nA * sizeof(double), hipMemcpyHostToDevice, s) == hipSuccess;
        }
        ok &= hipStreamSynchronize(s) == hipSuccess;
        if (!ok) return bail(fail(CBLP_EHIP, "uploading A^T failed"));
    }

    if (hipMemsetAsync(h->S_fx, 0, (size_t)n * 8, s) != hipSuccess)
        return bail(fail(CBLP_EHIP, "hipMemsetAsync failed"));
    if ((rc = reset_state(h, s))) return bail(rc);
    *out = h;
    return CBLP_OK;
}

void cblp_destroy(cblp_t h) { release(h); }

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
    int rc = check_params(h, p);
    if (rc) return rc;
    hipStream_t s = S(stream);
    if (trace && (rc = ensure_trace(h, std::max<int64_t>(iters, 1)))) return rc;
    if (iters == 0) {
        if (out) {
            out->iters = h->t;
            std::memset(out->trace, 0, sizeof(out->trace));
            out->seconds = 0.0;
            out->status = CBLP_OK;
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

int spfom_solve(cblp_t h, void* eta, const spfom_params* p, spfom_stats* out, void* stream)
{
    g_err.clear();
    if (!h || !eta || !out) return fail(CBLP_EINVAL, "NULL handle, eta or out");
    int rc = check_params(h, p);
    if (rc) return rc;
    if (p->max_iters < 0 || !(p->tol >= 0.0)) return fail(CBLP_EINVAL, "need max_iters >= 0 and tol >= 0");
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
    int rc = h->dtype == CBLP_F32 ? evaluate_impl<float>(h, eta, nullptr, s)
                                  : evaluate_impl<double>(h, eta, nullptr, s);
    if (rc) return rc;
    rc = fill_stats(h, out, s, h->trace);
    out->seconds = 0.0;
    return rc;
}

int cblp_sales(cblp_t h, const void* eta, double* S_out, double* u_out, void* seg_R_out,
               void* stream)
{
    g_err.clear();
    if (!h || !eta) return fail(CBLP_EINVAL, "NULL handle or eta");
    hipStream_t s = S(stream);
    int rc = h->dtype == CBLP_F32 ? evaluate_impl<float>(h, eta, seg_R_out, s)
                                  : evaluate_impl<double>(h, eta, seg_R_out, s);
    if (rc) return rc;
    if (S_out) HIP_TRY(hipMemcpyAsync(S_out, h->S_d, h->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (u_out) HIP_TRY(hipMemcpyAsync(u_out, h->u_d, h->m * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CBLP_OK;
}

}  // extern "C"

// Bid-price control with the global optimisation (GO) policy of Section 5.1,
// simulated for many independent runs at once on the market of Figure 4.
//
// Per batch of customers and run: products out of stock leave the offer (and
// the LP: their duals start at their revenue, so no assortment holds them);
// if at most K remain they are all offered, otherwise the batch's sales-based
// LP (its customers as segments, capacities = stock spread over the batches
// left) is re-solved by SPFOM from the previous batch's duals - all runs
// together as one batched solve - and the bid-price rule offers the products
// with r_j - eta_j >= 0, cut to the K largest margins.  Customers then choose
// under the basic attraction model (no-purchase attraction 1), one uniform
// each, and a product sells min(demand, stock) units.
//
// Kernels: k_lp_inputs (one block per run: capacities and dual steps),
// k_period (one block per run: offer, choices, sales, stock, revenue) and
// k_market_check (the handles hold the dense batch LP the simulation needs).
// Every integer decision is taken in FP64 from the same values in the same
// order as a plain sequential reading of the rule, so results are exact.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"
#include "handle.hpp"

namespace cblp {
namespace {

constexpr int kSimThreads = 1024;
constexpr int kSimMaxProducts = 8192;   // LDS flags of the offer selection
constexpr int kSimMaxOffer = 64;

#define GS_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return set_error(CBLP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// acc + a b rounded twice (no fused multiply-add), as a sequential FP64 sum
__device__ __noinline__ double add_product(double acc, double a, double b)
{
#pragma clang fp contract(off)
    return acc + a * b;
}

// c_j = inv_j / periods_left rounded once to T; tau_j = tau0 max_k r_k / c_j
// from the rounded capacities (zero capacity: the smallest positive one, or
// 1 if there is none), rounded once to T; a product out of stock has its dual
// raised to at least its revenue (eta nullable).  Block q handles run q.
template <typename T>
__global__ void __launch_bounds__(256) k_lp_inputs(int64_t n, const int64_t* inv,
                                                   double periods_left, double tau0, const T* r,
                                                   T* c, T* tau, T* eta)
{
    __shared__ double smax[256], smin[256];
    const int64_t off = (int64_t)blockIdx.x * n;
    double rmax = -INFINITY, cmin = INFINITY;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const T cj = (T)((double)inv[off + j] / periods_left);
        c[off + j] = cj;
        if (eta && inv[off + j] == 0 && eta[off + j] < r[off + j]) eta[off + j] = r[off + j];
        rmax = fmax(rmax, (double)r[off + j]);
        if ((double)cj > 0.0) cmin = fmin(cmin, (double)cj);
    }
    smax[threadIdx.x] = rmax;
    smin[threadIdx.x] = cmin;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
        }
        __syncthreads();
    }
    const double rm = smax[0];
    const double cm = smin[0] == INFINITY ? 1.0 : smin[0];
    const double num = tau0 * rm;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const double cj = (double)c[off + j];
        tau[off + j] = (T)(num / (cj > 0.0 ? cj : cm));
    }
}

// the larger of two offer candidates: larger margin, then lower index
__device__ __forceinline__ bool better(double m1, int j1, double m2, int j2)
{
    return j2 < 0 || (j1 >= 0 && (m1 > m2 || (m1 == m2 && j1 < j2)));
}

// One batch of every run; block q handles run q (kSimThreads threads).
template <typename T>
__global__ void __launch_bounds__(kSimThreads)
k_period(int64_t N, int64_t n, int K, const T* eta, const T* r, const T* prefs, const double* u,
         int64_t* inv, int32_t* offer, int64_t* sales, double* revenue, int32_t* in_stock)
{
    __shared__ unsigned char taken[kSimMaxProducts];
    __shared__ int sel[kSimMaxOffer];
    __shared__ int cnt[kSimMaxOffer];
    __shared__ int nsel, avail, stop;
    __shared__ double wm[kSimThreads / 64];
    __shared__ int wj[kSimThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t q = blockIdx.x;
    eta += q * n;
    r += q * n;
    inv += q * n;
    sales += q * n;
    prefs += q * N * n;
    u += q * N;
    if (tid == 0) {
        nsel = 0;
        avail = 0;
        stop = 0;
    }
    if (tid < kSimMaxOffer) cnt[tid] = 0;
    for (int64_t j = tid; j < n; j += kSimThreads) taken[j] = 0;
    __syncthreads();
    int mine = 0;
    for (int64_t j = tid; j < n; j += kSimThreads) mine += inv[j] > 0;
    if (mine) atomicAdd(&avail, mine);
    __syncthreads();
    if (avail <= K) {
        // every product in stock, ascending
        if (tid == 0) {
            int k = 0;
            for (int64_t j = 0; j < n; ++j)
                if (inv[j] > 0) sel[k++] = (int)j;
            nsel = k;
        }
    } else {
        // K rounds: the in-stock, not yet taken product of largest margin
        // r_j - eta_j >= 0 (ties: lower index)
        for (int k = 0; k < K; ++k) {
            double bm = 0.0;
            int bj = -1;
            for (int64_t j = tid; j < n; j += kSimThreads) {
                if (inv[j] <= 0 || taken[j]) continue;
                const double mj = (double)r[j] - (double)eta[j];
                if (mj >= 0.0 && better(mj, (int)j, bm, bj)) {
                    bm = mj;
                    bj = (int)j;
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double om = __shfl_down(bm, o, 64);
                const int oj = __shfl_down(bj, o, 64);
                if (better(om, oj, bm, bj)) {
                    bm = om;
                    bj = oj;
                }
            }
            if (lane == 0) {
                wm[wave] = bm;
                wj[wave] = bj;
            }
            __syncthreads();
            if (tid == 0) {
                for (int w = 1; w < kSimThreads / 64; ++w)
                    if (better(wm[w], wj[w], bm, bj)) {
                        bm = wm[w];
                        bj = wj[w];
                    }
                if (bj < 0) {
                    stop = 1;
                } else {
                    taken[bj] = 1;
                    sel[nsel++] = bj;
                }
            }
            __syncthreads();
            if (stop) break;
        }
        if (tid == 0) {
            // offered set in product order
            for (int a = 1; a < nsel; ++a) {
                const int x = sel[a];
                int b = a - 1;
                while (b >= 0 && sel[b] > x) {
                    sel[b + 1] = sel[b];
                    --b;
                }
                sel[b + 1] = x;
            }
        }
    }
    __syncthreads();
    const int ns = nsel;
    // choices: buy the first offered product whose running preference sum
    // exceeds u (1 + sum over the offer), else nothing
    for (int64_t i = tid; i < N; i += kSimThreads) {
        const T* row = prefs + i * n;
        double W = 1.0;
        for (int s = 0; s < ns; ++s) W += (double)row[sel[s]];
        const double x = u[i] * W;
        double cum = 0.0;
        for (int s = 0; s < ns; ++s) {
            cum += (double)row[sel[s]];
            if (x < cum) {
                atomicAdd(&cnt[s], 1);
                break;
            }
        }
    }
    for (int64_t j = tid; j < n; j += kSimThreads) sales[j] = 0;
    __syncthreads();
    if (tid == 0) {
        double rev = 0.0;
        for (int s = 0; s < ns; ++s) {
            const int j = sel[s];
            const int64_t sold = std::min<int64_t>((int64_t)cnt[s], inv[j]);
            inv[j] -= sold;
            sales[j] = sold;
            rev = add_product(rev, (double)r[j], (double)sold);
        }
        for (int s = 0; s < K; ++s) offer[q * K + s] = s < ns ? sel[s] : -1;
        revenue[q] = rev;
        avail = 0;
    }
    __syncthreads();
    if (in_stock) {
        mine = 0;
        for (int64_t j = tid; j < n; j += kSimThreads) mine += inv[j] > 0;
        if (mine) atomicAdd(&avail, mine);
        __syncthreads();
        if (tid == 0) in_stock[q] = avail;
    }
}

// The handle holds the batch LP the simulation reads: N rows that each list
// products 0..n-1 in order, no shadow attraction, and arrival rate and
// no-purchase attraction 1.
template <typename T>
__global__ void k_market_check(int64_t N, int64_t n, const int64_t* seg_ptr, const int32_t* idx,
                               const T* w, const T* v0, const T* lam, unsigned* flag)
{
    unsigned bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t l = tid; l <= N; l += stride) {
        if (seg_ptr[l] != l * n) bad = 1;
        if (l < N && (v0[l] != T(1) || lam[l] != T(1))) bad = 1;
    }
    for (int64_t e = tid; e < N * n; e += stride)
        if (idx[e] != (int32_t)(e % n) || w[e] != T(0)) bad = 1;
    if (bad) atomicOr(flag, 1u);
}

int check_sizes(int32_t runs, int64_t N, int64_t n, int32_t K, int32_t dtype)
{
    if (runs < 0 || N < 0 || n <= 0) return set_error(CBLP_EINVAL, "need runs >= 0, customers >= 0, products > 0");
    if (n > kSimMaxProducts)
        return set_error(CBLP_EINVAL, "at most " + std::to_string(kSimMaxProducts) + " products");
    if (K < 1 || K > kSimMaxOffer)
        return set_error(CBLP_EINVAL, "the offer limit K must be in [1, " + std::to_string(kSimMaxOffer) + "]");
    if (dtype != CBLP_F32 && dtype != CBLP_F64) return set_error(CBLP_EINVAL, "dtype must be CBLP_F32 or CBLP_F64");
    return CBLP_OK;
}

template <typename T>
hipError_t launch_lp_inputs(int32_t runs, int64_t n, const int64_t* inv, int64_t periods_left,
                            double tau0, const void* r, void* c, void* tau, void* eta,
                            hipStream_t s)
{
    if (runs > 0)
        hipLaunchKernelGGL(k_lp_inputs<T>, dim3(runs), dim3(256), 0, s, n, inv,
                           (double)periods_left, tau0, (const T*)r, (T*)c, (T*)tau, (T*)eta);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_period(int32_t runs, int64_t N, int64_t n, int32_t K, const void* eta,
                         const void* r, const void* prefs, const double* u, int64_t* inv,
                         int32_t* offer, int64_t* sales, double* revenue, int32_t* in_stock,
                         hipStream_t s)
{
    if (runs > 0)
        hipLaunchKernelGGL(k_period<T>, dim3(runs), dim3(kSimThreads), 0, s, N, n, K,
                           (const T*)eta, (const T*)r, (const T*)prefs, u, inv, offer, sales,
                           revenue, in_stock);
    return hipGetLastError();
}

}  // namespace
}  // namespace cblp

using namespace cblp;

extern "C" {

int gosim_lp_inputs(int32_t runs, int64_t n, const int64_t* inv, int64_t periods_left,
                    double tau0, const void* r, void* c, void* tau, void* eta, int32_t dtype,
                    void* stream)
{
    set_error(CBLP_OK, "");
    int rc = check_sizes(runs, 0, n, 1, dtype);
    if (rc) return rc;
    if (periods_left < 1) return set_error(CBLP_EINVAL, "periods_left must be >= 1");
    if (!(tau0 > 0.0)) return set_error(CBLP_EINVAL, "tau0 must be > 0");
    if (runs > 0 && (!inv || !r || !c || !tau)) return set_error(CBLP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    GS_TRY(dtype == CBLP_F32 ? launch_lp_inputs<float>(runs, n, inv, periods_left, tau0, r, c, tau, eta, s)
                             : launch_lp_inputs<double>(runs, n, inv, periods_left, tau0, r, c, tau, eta, s));
    return CBLP_OK;
}

int gosim_period(int32_t runs, int64_t N, int64_t n, int32_t K, const void* eta, const void* r,
                 const void* prefs, const double* u, int64_t* inv, int32_t* offer,
                 int64_t* sales, double* revenue, int32_t* in_stock, int32_t dtype, void* stream)
{
    set_error(CBLP_OK, "");
    int rc = check_sizes(runs, N, n, K, dtype);
    if (rc) return rc;
    if (runs > 0 && (!eta || !r || (N > 0 && (!prefs || !u)) || !inv || !offer || !sales || !revenue))
        return set_error(CBLP_EINVAL, "NULL array");
    hipStream_t s = (hipStream_t)stream;
    GS_TRY(dtype == CBLP_F32
               ? launch_period<float>(runs, N, n, K, eta, r, prefs, u, inv, offer, sales, revenue, in_stock, s)
               : launch_period<double>(runs, N, n, K, eta, r, prefs, u, inv, offer, sales, revenue, in_stock, s));
    return CBLP_OK;
}

int gosim_run(cblp_batch_t b, int32_t periods, int32_t K, const void* prefs, const double* u,
              const void* r, int64_t* inv, void* eta, void* tau_work, const spfom_params* p,
              double tau0, int32_t* offers, int64_t* sales, double* revenue, int64_t* lp_iters,
              double* lp_gap, void* stream)
{
    set_error(CBLP_OK, "");
    if (!b || !p) return set_error(CBLP_EINVAL, "NULL batch or params");
    const std::vector<cblp_instance*>& hs = batch_handles(b);
    const int32_t runs = (int32_t)hs.size();
    if (runs == 0) return CBLP_OK;
    const cblp_instance* h0 = hs[0];
    const int64_t N = h0->L, n = h0->n;
    const int32_t dtype = h0->dtype;
    int rc = check_sizes(runs, N, n, K, dtype);
    if (rc) return rc;
    if (periods < 0) return set_error(CBLP_EINVAL, "periods must be >= 0");
    if (!(tau0 > 0.0)) return set_error(CBLP_EINVAL, "tau0 must be > 0");
    if (!prefs || !u || !r || !inv || !eta || !tau_work || !offers || !sales || !revenue)
        return set_error(CBLP_EINVAL, "NULL array");
    const size_t esz = h0->esz;
    const size_t vrun = (size_t)N * (size_t)n * esz;
    for (int q = 0; q < runs; ++q) {
        const cblp_instance* h = hs[q];
        if (h->L != N || h->n != n || h->m != n || h->a_ptr || h->dtype != dtype || h->nnz != N * n)
            return set_error(CBLP_EINVAL, "run " + std::to_string(q) + ": every handle must hold "
                             "N customers over the same n products (A = I, one dtype)");
        if ((const char*)h->v != (const char*)h0->v + q * vrun ||
            (const char*)h->c != (const char*)h0->c + q * n * esz ||
            (const char*)h->r != (const char*)r + q * n * esz)
            return set_error(CBLP_EINVAL, "run " + std::to_string(q) + ": handle q must read v, c "
                             "and r at offset q of one [runs x ...] array each (r: the r argument)");
    }
    hipStream_t s = (hipStream_t)stream;
    unsigned* dflags = nullptr;
    int32_t* d_stock = nullptr;
    if (hipMalloc((void**)&dflags, (size_t)runs * sizeof(unsigned)) != hipSuccess ||
        hipMalloc((void**)&d_stock, (size_t)runs * sizeof(int32_t)) != hipSuccess) {
        (void)hipGetLastError();
        if (dflags) (void)hipFree(dflags);
        return set_error(CBLP_ENOMEM, "hipMalloc of the simulation's flags failed");
    }
    std::vector<unsigned> flags((size_t)runs);
    std::vector<int32_t> stock((size_t)runs);
    std::vector<int64_t> hinv((size_t)runs * n);
    std::vector<int32_t> take((size_t)runs);
    std::vector<spfom_stats> outs((size_t)runs);
    std::vector<void*> etas((size_t)runs);
    std::vector<const void*> taus((size_t)runs);
    for (int q = 0; q < runs; ++q) {
        etas[q] = (char*)eta + q * n * esz;
        taus[q] = (const char*)tau_work + q * n * esz;
    }
    auto run = [&]() -> int {
        // the handles must hold the dense batch LP
        GS_TRY(hipMemsetAsync(dflags, 0, (size_t)runs * sizeof(unsigned), s));
        for (int q = 0; q < runs; ++q) {
            const cblp_instance* h = hs[q];
            const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (N * n + 255) / 256));
            if (dtype == CBLP_F32)
                hipLaunchKernelGGL(k_market_check<float>, dim3(blocks), dim3(256), 0, s, N, n,
                                   h->seg_ptr, h->idx, (const float*)h->w, (const float*)h->v0,
                                   (const float*)h->lam, dflags + q);
            else
                hipLaunchKernelGGL(k_market_check<double>, dim3(blocks), dim3(256), 0, s, N, n,
                                   h->seg_ptr, h->idx, (const double*)h->w, (const double*)h->v0,
                                   (const double*)h->lam, dflags + q);
            GS_TRY(hipGetLastError());
        }
        GS_TRY(hipMemcpyAsync(flags.data(), dflags, (size_t)runs * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        GS_TRY(hipMemcpyAsync(hinv.data(), inv, hinv.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        GS_TRY(hipStreamSynchronize(s));
        for (int q = 0; q < runs; ++q)
            if (flags[q])
                return set_error(CBLP_EINVAL, "run " + std::to_string(q) + ": the handle is not the dense "
                                 "batch LP (rows listing every product in order, w = 0, v0 = lambda = 1)");
        for (int q = 0; q < runs; ++q) {
            int k = 0;
            for (int64_t j = 0; j < n; ++j) k += hinv[(size_t)q * n + j] > 0;
            stock[q] = k;
        }
        for (int32_t t = 0; t < periods; ++t) {
            // this batch's LP: capacities, steps and the customers' preferences
            GS_TRY(dtype == CBLP_F32
                       ? launch_lp_inputs<float>(runs, n, inv, periods - t, tau0, r, (void*)h0->c, tau_work, eta, s)
                       : launch_lp_inputs<double>(runs, n, inv, periods - t, tau0, r, (void*)h0->c, tau_work, eta, s));
            GS_TRY(hipMemcpyAsync((void*)h0->v, (const char*)prefs + (size_t)t * runs * vrun,
                                  (size_t)runs * vrun, hipMemcpyDeviceToDevice, s));
            int any = 0;
            for (int q = 0; q < runs; ++q) {
                take[q] = stock[q] > K;
                any += take[q];
            }
            if (any) {
                GS_TRY(hipMemsetAsync(dflags, 0, (size_t)runs * sizeof(unsigned), s));
                for (int q = 0; q < runs; ++q) {
                    if (!take[q]) continue;
                    int e = refresh_launch(hs[q], dflags + q, s);
                    if (e) return e;
                }
                GS_TRY(hipMemcpyAsync(flags.data(), dflags, (size_t)runs * sizeof(unsigned), hipMemcpyDeviceToHost, s));
                GS_TRY(hipStreamSynchronize(s));
                for (int q = 0; q < runs; ++q)
                    if (take[q] && flags[q])
                        return set_error(CBLP_EINVAL, "batch " + std::to_string(t) + ", run " + std::to_string(q) +
                                         ": " + validation_message(flags[q]));
                int e = cblp_batch_mask(b, take.data());
                if (e) return e;
                e = spfom_batch_solve(b, etas.data(), taus.data(), p, outs.data(), stream);
                if (e == CBLP_ENONFINITE || (e && e != CBLP_ENOTCONVERGED)) return e;
                set_error(CBLP_OK, "");
            }
            for (int q = 0; q < runs; ++q) {
                if (lp_iters) lp_iters[(size_t)t * runs + q] = take[q] ? outs[q].iters : 0;
                if (lp_gap) lp_gap[(size_t)t * runs + q] = take[q] ? outs[q].trace[SPFOM_TR_GAP] : 0.0;
            }
            GS_TRY(dtype == CBLP_F32
                       ? launch_period<float>(runs, N, n, K, eta, r, (const char*)prefs + (size_t)t * runs * vrun,
                                              u + (size_t)t * runs * N, inv, offers + (size_t)t * runs * K,
                                              sales + (size_t)t * runs * n, revenue + (size_t)t * runs,
                                              d_stock, s)
                       : launch_period<double>(runs, N, n, K, eta, r, (const char*)prefs + (size_t)t * runs * vrun,
                                               u + (size_t)t * runs * N, inv, offers + (size_t)t * runs * K,
                                               sales + (size_t)t * runs * n, revenue + (size_t)t * runs,
                                               d_stock, s));
            GS_TRY(hipMemcpyAsync(stock.data(), d_stock, (size_t)runs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
            GS_TRY(hipStreamSynchronize(s));
        }
        return CBLP_OK;
    };
    rc = run();
    (void)cblp_batch_mask(b, nullptr);
    (void)hipStreamSynchronize(s);
    (void)hipFree(dflags);
    (void)hipFree(d_stock);
    return rc;
}

}  // extern "C"

// Instance validation, the library's sorted copy of the instance, arrival-rate
// bounds and the price step.
#include "handle.hpp"

#include <algorithm>

namespace cblp {
namespace {

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
        const int32_t j = idx[q];
        if (j < 0 || j >= n) bad |= V_IDX;
        const T a = v[q], b = w[q];
        if (!(a > T(0)) || !isfinite(a)) bad |= V_V;
        if (!(b >= T(0)) || !(b < a)) bad |= V_W;
    }
    for (int64_t l = tid; l < L; l += stride) {
        const T a = v0[l], b = lam[l];
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
        const T x = c[i];
        if (!(x >= T(0)) || !isfinite(x)) bad |= V_C;
    }
    if (a_ptr) {
        if (tid == 0 && (a_ptr[0] != 0 || a_ptr[n] != nnzA)) bad |= V_APTR;
        for (int64_t q = tid; q < nnzA; q += stride) {
            const int32_t i = a_idx[q];
            if (i < 0 || i >= m) bad |= V_AIDX;
            const T x = a_val[q];
            if (!(x >= T(0)) || !isfinite(x)) bad |= V_AVAL;
        }
    }
    if (bad) atomicOr(flags, bad);
}

// Block partial sum and maximum of the arrival rates: every product's sales
// are at most sum_l lambda_l and one segment's sales of one product at most
// max_l lambda_l, which set the fixed-point scales of the sales sums.
template <typename T>
__global__ void k_prepare(int64_t L, const T* lam, double* lam_part)
{
    __shared__ double sh[256], mx[256];
    double acc = 0.0, hi = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double x = (double)lam[l];
        acc += x;
        hi = x > hi ? x : hi;
    }
    sh[threadIdx.x] = acc;
    mx[threadIdx.x] = hi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[threadIdx.x] += sh[threadIdx.x + o];
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        lam_part[2 * blockIdx.x] = sh[0];
        lam_part[2 * blockIdx.x + 1] = mx[0];
    }
}

// Copy the caller's CSR into the library's layout: position p takes
// segment perm[p]; entries keep their order within a row; den = v - w;
// product ids become pnew[id] (nullable: ids kept).
template <typename T>
__global__ void k_relayout(int64_t L, const int64_t* seg_ptr, const int32_t* idx, const T* v,
                           const T* w, const T* v0, const T* lam, const int32_t* perm,
                           const int32_t* pnew, const int64_t* ptr, int32_t* idx2, T* v2,
                           T* den2, T* vt0, T* lam2, T* Rwarm, T* v0c)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = perm[p];
        const int64_t b = seg_ptr[l], k = seg_ptr[l + 1] - b, d = ptr[p];
        double s = (double)v0[l];
        for (int64_t q = 0; q < k; ++q) {
            const T x = v[b + q], y = w[b + q];
            const int32_t id = idx[b + q];
            idx2[d + q] = pnew ? pnew[id] : id;
            v2[d + q] = x;
            den2[d + q] = x - y;
            s += (double)y;
        }
        vt0[p] = (T)s;
        lam2[p] = lam[l];
        v0c[p] = v0[l];
        Rwarm[p] = T(0);
    }
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T val)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// Slot-major copy: the eight rows of wave-tile w = p / 8 occupy woff[w] ..
// woff[w + 1] (64 entries per slot); entry t of row p goes to slot t / 8 at
// lane 8 (p % 8) + t % 8.  Unused places keep (product 0, v 0, den 1).
// G lanes per row (8, 4: quad layout, 2: pair layout): rows Rw..Rw+R-1 per
// wave-tile (R = 64 / G), entry t of row p at slot t / G, lane G (p % R) + t % G.
template <typename T, typename IdxT, int G>
__global__ void k_relayout_slots(int64_t L, const int64_t* ptr, const int32_t* idx2,
                                 const T* v2, const T* den2, const int64_t* woff, IdxT* idx3,
                                 T* v3, T* den3)
{
    constexpr int R = 64 / G;   // rows per wave-tile
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < L;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = ptr[p], k = ptr[p + 1] - b;
        const int64_t base = woff[p / R] + G * (p % R);
        for (int64_t t = 0; t < k; ++t) {
            const int64_t d = base + 64 * (t / G) + (t % G);
            idx3[d] = (IdxT)idx2[b + t];
            v3[d] = v2[b + t];
            den3[d] = den2[b + t];
        }
    }
}

// New attractions and capacities on the structure of creation: re-read the
// caller's v and w (the row pointers, product ids, arrival rates and
// no-purchase attractions are those the copies were built from) into the
// sorted copy (v2, den2, vt0 as k_relayout writes them) and into the
// slot-major copy of whichever part holds each position (the places
// k_relayout_slots gives them); warm starts go back to zero.  Flags invalid
// v, w and c as k_validate does.
template <typename T>
__global__ void k_refresh(int64_t L, int64_t m, const int64_t* seg_ptr, const T* v, const T* w,
                          const T* v0, const T* c, const int32_t* perm, const int64_t* ptr2,
                          const int64_t* woff, int64_t pair_end, int64_t quad_end,
                          int64_t woff_q, int64_t woff_b, T* v2, T* den2, T* vt0, T* Rwarm,
                          T* v3, T* den3, unsigned* flags)
{
    unsigned bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t p = tid; p < L; p += stride) {
        const int64_t l = perm[p];
        const int64_t b = seg_ptr[l], k = seg_ptr[l + 1] - b, d = ptr2[p];
        int64_t G, base;
        if (p < pair_end) {
            G = 2;
            base = woff[p / 32] + 2 * (p % 32);
        } else if (p < quad_end) {
            const int64_t q = p - pair_end;
            G = 4;
            base = woff[woff_q + q / 16] + 4 * (q % 16);
        } else {
            const int64_t q = p - quad_end;
            G = kGroup;
            base = woff[woff_b + q / kGroup] + kGroup * (q % kGroup);
        }
        double s = (double)v0[l];
        for (int64_t t = 0; t < k; ++t) {
            const T x = v[b + t], y = w[b + t];
            if (!(x > T(0)) || !isfinite(x)) bad |= V_V;
            if (!(y >= T(0)) || !(y < x)) bad |= V_W;
            v2[d + t] = x;
            den2[d + t] = x - y;
            s += (double)y;
            const int64_t e = base + 64 * (t / G) + t % G;
            v3[e] = x;
            den3[e] = x - y;
        }
        vt0[p] = (T)s;
        Rwarm[p] = T(0);
    }
    for (int64_t i = tid; i < m; i += stride) {
        const T x = c[i];
        if (!(x >= T(0)) || !isfinite(x)) bad |= V_C;
    }
    if (bad) atomicOr(flags, bad);
}

// Degrees of the products [lo, lo + kDegBins): per-block LDS counts over the
// block's share of the entries, then one global atomic per nonzero bin.
constexpr int kDegBins = 16384;

__global__ void __launch_bounds__(1024) k_degree(int64_t nnz, const int32_t* idx, int64_t lo,
                                                 int64_t hi, unsigned long long* deg)
{
    __shared__ unsigned cnt[kDegBins];
    for (int j = threadIdx.x; j < kDegBins; j += blockDim.x) cnt[j] = 0u;
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = idx[e];
        if (id >= lo && id < hi) atomicAdd(&cnt[id - lo], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < kDegBins && lo + j < hi; j += blockDim.x)
        if (cnt[j]) atomicAdd(&deg[lo + j], (unsigned long long)cnt[j]);
}

// rho_j = r_j - sum_i a_ij eta_i  (identity: r_j - eta_j), stored at the
// library's product id pnew[j] (nullable: j)
template <typename T>
__global__ void k_prices(int64_t n, const T* r, const T* eta, const int64_t* a_ptr,
                         const int32_t* a_idx, const T* a_val, const int32_t* pnew, T* rho)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        T x = r[j];
        if (!a_ptr) {
            x -= eta[j];
        } else {
            for (int64_t q = a_ptr[j]; q < a_ptr[j + 1]; ++q) x -= a_val[q] * eta[a_idx[q]];
        }
        rho[pnew ? pnew[j] : j] = x;
    }
}

}  // namespace

hipError_t launch_degree(int64_t nnz, const int32_t* idx, int64_t n, unsigned long long* deg,
                         hipStream_t s)
{
    hipError_t e = hipMemsetAsync(deg, 0, (size_t)n * 8, s);
    if (e != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>(1024, std::max<int64_t>(1, (nnz + 1023) / 1024));
    for (int64_t lo = 0; lo < n; lo += kDegBins)
        hipLaunchKernelGGL(k_degree, dim3((unsigned)blocks), dim3(1024), 0, s, nnz, idx, lo,
                           std::min<int64_t>(n, lo + kDegBins), deg);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_validate(int64_t L, int64_t n, int64_t m, int64_t nnz, int64_t nnzA,
                           const int64_t* seg_ptr, const int32_t* idx, const void* v,
                           const void* w, const void* v0, const void* lam, const void* r,
                           const void* c, const int64_t* a_ptr, const int32_t* a_idx,
                           const void* a_val, unsigned* flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_validate<T>, dim3(1024), dim3(256), 0, s, L, n, m, nnz, nnzA, seg_ptr,
                       idx, (const T*)v, (const T*)w, (const T*)v0, (const T*)lam,
                       (const T*)r, (const T*)c, a_ptr, a_idx, (const T*)a_val, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prepare(int64_t L, const void* lam, double* lam_part, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_prepare<T>, dim3(blocks), dim3(256), 0, s, L, (const T*)lam, lam_part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_relayout(int64_t L, const int64_t* seg_ptr, const int32_t* idx,
                           const void* v, const void* w, const void* v0, const void* lam,
                           const int32_t* perm, const int32_t* pnew, const int64_t* ptr,
                           int32_t* idx2, void* v2, void* den2, void* vt0, void* lam2, void* Rwarm,
                           void* v0c, hipStream_t s)
{
    hipLaunchKernelGGL(k_relayout<T>, dim3(2048), dim3(256), 0, s, L, seg_ptr, idx,
                       (const T*)v, (const T*)w, (const T*)v0, (const T*)lam, perm, pnew, ptr, idx2,
                       (T*)v2, (T*)den2, (T*)vt0, (T*)lam2, (T*)Rwarm, (T*)v0c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_relayout_slots(int64_t L, const int64_t* ptr, const int32_t* idx2,
                                 const void* v2, const void* den2, const int64_t* woff,
                                 int64_t entries, void* idx3, bool idx16, int G, void* v3,
                                 void* den3, hipStream_t s)
{
    if (idx16)
        hipLaunchKernelGGL(k_fill<uint16_t>, dim3(1024), dim3(256), 0, s, (uint16_t*)idx3, entries,
                           (uint16_t)0);
    else
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(1024), dim3(256), 0, s, (int32_t*)idx3, entries, 0);
    hipLaunchKernelGGL(k_fill<T>, dim3(1024), dim3(256), 0, s, (T*)v3, entries, T(0));
    hipLaunchKernelGGL(k_fill<T>, dim3(1024), dim3(256), 0, s, (T*)den3, entries, T(1));
    if (L > 0 && idx16 && G == 2)
        hipLaunchKernelGGL((k_relayout_slots<T, uint16_t, 2>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (uint16_t*)idx3, (T*)v3,
                           (T*)den3);
    else if (L > 0 && G == 2)
        hipLaunchKernelGGL((k_relayout_slots<T, int32_t, 2>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (int32_t*)idx3, (T*)v3,
                           (T*)den3);
    else if (L > 0 && idx16 && G == 4)
        hipLaunchKernelGGL((k_relayout_slots<T, uint16_t, 4>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (uint16_t*)idx3, (T*)v3,
                           (T*)den3);
    else if (L > 0 && G == 4)
        hipLaunchKernelGGL((k_relayout_slots<T, int32_t, 4>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (int32_t*)idx3, (T*)v3,
                           (T*)den3);
    else if (L > 0 && idx16)
        hipLaunchKernelGGL((k_relayout_slots<T, uint16_t, 8>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (uint16_t*)idx3, (T*)v3,
                           (T*)den3);
    else if (L > 0)
        hipLaunchKernelGGL((k_relayout_slots<T, int32_t, 8>), dim3(2048), dim3(256), 0, s, L, ptr,
                           idx2, (const T*)v2, (const T*)den2, woff, (int32_t*)idx3, (T*)v3,
                           (T*)den3);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_refresh(const cblp_instance* h, unsigned* flags, hipStream_t s)
{
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(2048, (h->L + 255) / 256));
    hipLaunchKernelGGL(k_refresh<T>, dim3((unsigned)blocks), dim3(256), 0, s, h->L, h->m,
                       h->seg_ptr, (const T*)h->v, (const T*)h->w, (const T*)h->v0,
                       (const T*)h->c, h->perm, h->ptr2, h->woff, h->pair_end, h->quad_end,
                       h->woff_q, h->woff_b, (T*)h->v2, (T*)h->den2, (T*)h->vt0, (T*)h->Rwarm,
                       (T*)h->v3, (T*)h->den3, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prices(int64_t n, const void* r, const void* eta, const int64_t* a_ptr,
                         const int32_t* a_idx, const void* a_val, const int32_t* pnew, void* rho,
                         hipStream_t s)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_prices<T>, dim3((unsigned)(blocks < 1 ? 1 : blocks > 4096 ? 4096 : blocks)),
                       dim3(256), 0, s, n, (const T*)r, (const T*)eta, a_ptr, a_idx,
                       (const T*)a_val, pnew, (T*)rho);
    return hipGetLastError();
}

#define CBLP_INST(T)                                                                           \
    template hipError_t launch_validate<T>(int64_t, int64_t, int64_t, int64_t, int64_t,        \
                                           const int64_t*, const int32_t*, const void*,       \
                                           const void*, const void*, const void*, const void*, \
                                           const void*, const int64_t*, const int32_t*,        \
                                           const void*, unsigned*, hipStream_t);               \
    template hipError_t launch_prepare<T>(int64_t, const void*, double*, int, hipStream_t);    \
    template hipError_t launch_prices<T>(int64_t, const void*, const void*, const int64_t*,    \
                                         const int32_t*, const void*, const int32_t*, void*,   \
                                         hipStream_t);                                         \
    template hipError_t launch_relayout<T>(int64_t, const int64_t*, const int32_t*,            \
                                           const void*, const void*, const void*, const void*, \
                                           const int32_t*, const int32_t*, const int64_t*,     \
                                           int32_t*, void*, void*, void*, void*, void*, void*, \
                                           hipStream_t);                                       \
    template hipError_t launch_relayout_slots<T>(int64_t, const int64_t*, const int32_t*,      \
                                                 const void*, const void*, const int64_t*,     \
                                                 int64_t, void*, bool, int, void*, void*,        \
                                                 hipStream_t);                                 \
    template hipError_t launch_refresh<T>(const cblp_instance*, unsigned*, hipStream_t);
CBLP_INST(float)
CBLP_INST(double)
#undef CBLP_INST

}  // namespace cblp

// cblp_gap_static: the dual bound D(eta), the revenue P and the product
// sales S of one best-response pass, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  It takes the
// instance arrays themselves instead of a handle (cblp_create allocates) and
// keeps every intermediate in one file-scope device array, `scratch`:
//
//   [0, kHdr)            header: fixed-point scale, its inverse, error bits
//   lam_part             [kLamBlocks x 2] partial sums / maxima of lambda
//   zpart                [kSegBlocks] partial sums of lambda R*
//   fpart                [fold blocks x 2] partial sums of r.S and c.eta
//   rho                  [n] reduced revenues (instance dtype, 8-byte slots)
//   S_fx                 [n] 64-bit fixed-point sales sums
//
// The passes are the library's (same per-segment arithmetic, same
// fixed-point scale), run over the caller's CSR as given: one 8-lane group
// per segment, Dinkelbach from R = 0, sales summed as 64-bit integers.  Every
// buffer is cleared by a kernel (no memset), nothing is read back, and the
// call allocates nothing.  Each GPU holds its own copy of `scratch`; calls on
// one GPU share it, so calls that overlap on one GPU race.
#include <algorithm>
#include <mutex>
#include <string>

#include "segment_core.hpp"

namespace cblp {
namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;   // 8 MiB per GPU
constexpr int kLamBlocks = 256;                     // as the handle's lambda reduction
constexpr int kSegBlocks = 1024;
constexpr size_t kHdr = 256;
constexpr size_t kFixed = kHdr + kLamBlocks * 16 + kSegBlocks * 8;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

struct Hdr {
    double fx, inv_fx;
    unsigned err;   // bit 0: arrival rates too large; bit 1: bad index or row pointer
};

// the largest n whose partials, prices and sums fit after the fixed part
constexpr int64_t max_products()
{
    // per product: 8 (rho slot) + 8 (S_fx) + 16 / 256 (fold partials), rounded up
    return (int64_t)((kScratchBytes - kFixed - 1024) / 17);
}

struct Layout {
    Hdr* hdr;
    double* lam_part;
    double* zpart;
    double* fpart;
    void* rho;
    unsigned long long* S_fx;
};

Layout layout(void* base, int64_t n, int64_t m)
{
    char* p = (char*)base;
    Layout o;
    o.hdr = (Hdr*)p;
    o.lam_part = (double*)(p + kHdr);
    o.zpart = (double*)(p + kHdr + kLamBlocks * 16);
    o.fpart = (double*)(p + kFixed);
    const int64_t fb = (std::max(n, m) + 255) / 256;   // blocks of k_na_fold
    size_t off = kFixed + (size_t)fb * 16;
    off = (off + 255) / 256 * 256;
    o.rho = p + off;
    off += (size_t)n * 8;
    o.S_fx = (unsigned long long*)(p + off);
    return o;
}

template <typename T>
__global__ void __launch_bounds__(256) k_na_lam(int64_t L, const T* lam, double* part)
{
    __shared__ double sh[256], mx[256];
    double acc = 0.0, hi = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
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
        part[2 * blockIdx.x] = sh[0];
        part[2 * blockIdx.x + 1] = mx[0];
    }
}

// prices and cleared sums; block 0 also forms the fixed-point scale the way
// cblp_create does (every 64-bit sum below 2^61, an FP32 quantum below 2^30)
template <typename T>
__global__ void __launch_bounds__(256) k_na_setup(int64_t n, const T* r, const T* eta,
                                                  const int64_t* a_ptr, const int32_t* a_idx,
                                                  const T* a_val, int64_t m, Layout o)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) {
        T x = r[j];
        if (!a_ptr) {
            x -= eta[j];
        } else {
            for (int64_t q = a_ptr[j]; q < a_ptr[j + 1]; ++q) {
                const int32_t i = a_idx[q];
                if (i < 0 || (int64_t)i >= m) {
                    atomicOr(&o.hdr->err, 2u);
                    continue;
                }
                x -= a_val[q] * eta[i];
            }
        }
        ((T*)o.rho)[j] = x;
        o.S_fx[j] = 0ull;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double tot = 0.0, hi = 0.0;
        for (int q = 0; q < kLamBlocks; ++q) {
            tot += o.lam_part[2 * q];
            hi = fmax(hi, o.lam_part[2 * q + 1]);
        }
        int e_tot = 0, e_hi = 0;
        frexp(tot + 1.0, &e_tot);
        frexp(hi, &e_hi);
        int bits = min(60, 61 - e_tot);
        if (sizeof(T) == 4) bits = min(bits, 30 - e_hi);
        if (bits < 8) atomicOr(&o.hdr->err, 1u);
        o.hdr->fx = ldexp(1.0, bits);
        o.hdr->inv_fx = ldexp(1.0, -bits);
    }
}

// the per-segment step over the caller's CSR (the library's arithmetic)
template <typename T>
__global__ void __launch_bounds__(256) k_na_segments(int64_t L, int64_t n, const int64_t* seg_ptr,
                                                     const int32_t* idx, const T* v, const T* w,
                                                     const T* v0, const T* lam, Layout o)
{
    __shared__ double zsh[4];
    const int g = threadIdx.x & (kGroup - 1);
    const int lane = threadIdx.x & 63;
    const T* rho = (const T*)o.rho;
    const T fx = (T)o.hdr->fx;
    double zacc = 0.0;
    for (int64_t l = (int64_t)blockIdx.x * 32 + threadIdx.x / kGroup; l < L;
         l += (int64_t)gridDim.x * 32) {
        const int64_t b = seg_ptr[l], e = seg_ptr[l + 1];
        if (e < b || b < 0) {
            if (g == 0) atomicOr(&o.hdr->err, 2u);
            continue;
        }
        const int k = (int)(e - b);
        bool bad = false;
        double s = (double)v0[l];
        for (int t = 0; t < k; ++t) s += (double)w[b + t];
        const T vt0 = (T)s;
        for (int t = g; t < k; t += kGroup) bad = bad || idx[b + t] < 0 || (int64_t)idx[b + t] >= n;
        if (((__ballot(bad) >> (lane & 56)) & 0xFFull) != 0ull) {
            if (g == 0) atomicOr(&o.hdr->err, 2u);
            continue;
        }
        auto full = [&](T R, T& N, T& Dn) {
            T n_ = T(0), d_ = T(0);
            for (int t = g; t < k; t += kGroup) {
                const T x = v[b + t];
                const T nn = rho[idx[b + t]] * x;
                const T dd = x - w[b + t];
                const T wt = nn > R * dd ? T(1) : T(0);
                n_ = seg::fmadd(wt, nn, n_);
                d_ = seg::fmadd(wt, dd, d_);
            }
            N = seg::group_sum(n_);
            Dn = seg::group_sum(d_);
        };
        auto changed = [&](T R, T Rn) {
            bool c = false;
            for (int t = g; t < k; t += kGroup) {
                const T x = v[b + t];
                const T nn = rho[idx[b + t]] * x;
                const T dd = x - w[b + t];
                c = c || ((nn > Rn * dd) != (nn > R * dd));
            }
            return ((__ballot(c) >> (lane & 56)) & 0xFFull) != 0ull;
        };
        T R = T(0), N, Dn;
        full(R, N, Dn);
        T Rs = N > T(0) ? seg::ratio(N, vt0 + Dn) : T(0);
        T pR = R, pN = N, pD = Dn, pRs = Rs;
        bool diff = false;
        const int cap = kGroup * ((k + kGroup - 1) / kGroup) + 1;
        for (int round = 0; round <= cap; ++round) {
            diff = changed(R, Rs);
            if (!diff) break;
            pR = R;
            pN = N;
            pD = Dn;
            pRs = Rs;
            R = Rs;
            full(R, N, Dn);
            Rs = N > T(0) ? seg::ratio(N, vt0 + Dn) : T(0);
        }
        if (diff && changed(R, Rs) && pRs > Rs) {   // alternating: the set of larger ratio
            R = pR;
            Dn = pD;
            Rs = pRs;
        }
        const T lamD = seg::ratio(lam[l], vt0 + Dn) * fx;
        for (int t = g; t < k; t += kGroup) {
            const T x = v[b + t];
            const int32_t j = idx[b + t];
            if (rho[j] * x > R * (x - w[b + t])) atomicAdd(&o.S_fx[j], seg::quantum(lamD, x));
        }
        if (g == 0) zacc += (double)lam[l] * (double)Rs;
    }
    for (int off = 32; off > 0; off >>= 1) zacc += __shfl_down(zacc, off, 64);
    if (lane == 0) zsh[threadIdx.x >> 6] = zacc;
    __syncthreads();
    if (threadIdx.x == 0) o.zpart[blockIdx.x] = ((zsh[0] + zsh[1]) + zsh[2]) + zsh[3];
}

// S_j, and per block the partial sums of r . S and c . eta
template <typename T>
__global__ void __launch_bounds__(256) k_na_fold(int64_t n, int64_t m, const T* r, const T* c,
                                                 const T* eta, double* S_out, Layout o)
{
    __shared__ double sp[4], sc[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double p = 0.0, ce = 0.0;
    if (j < n) {
        const double sj = (double)(long long)o.S_fx[j] * o.hdr->inv_fx;
        if (S_out) S_out[j] = sj;
        p = (double)r[j] * sj;
    }
    if (j < m) ce = (double)c[j] * (double)eta[j];
    for (int off = 32; off > 0; off >>= 1) {
        p += __shfl_down(p, off, 64);
        ce += __shfl_down(ce, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sp[threadIdx.x >> 6] = p;
        sc[threadIdx.x >> 6] = ce;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        o.fpart[2 * blockIdx.x] = ((sp[0] + sp[1]) + sp[2]) + sp[3];
        o.fpart[2 * blockIdx.x + 1] = ((sc[0] + sc[1]) + sc[2]) + sc[3];
    }
}

__global__ void __launch_bounds__(256) k_na_final(int nz, int nf, Layout o, double* bounds)
{
    __shared__ double s3[3][256];
    double z = 0.0, p = 0.0, ce = 0.0;
    for (int q = threadIdx.x; q < nz; q += 256) z += o.zpart[q];
    for (int q = threadIdx.x; q < nf; q += 256) {
        p += o.fpart[2 * q];
        ce += o.fpart[2 * q + 1];
    }
    s3[0][threadIdx.x] = z;
    s3[1][threadIdx.x] = p;
    s3[2][threadIdx.x] = ce;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 3; ++k) s3[k][threadIdx.x] += s3[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool ok = o.hdr->err == 0u;
        bounds[0] = ok ? s3[2][0] + s3[0][0] : NAN;   // D = c . eta + sum lambda R*
        bounds[1] = ok ? s3[1][0] : NAN;              // P = r . S
    }
}

__global__ void k_na_clear(Layout o) { o.hdr->err = 0u; }

template <typename T>
int run(int64_t L, int64_t n, int64_t m, const int64_t* seg_ptr, const int32_t* idx,
        const void* v, const void* w, const void* v0, const void* lam, const void* r,
        const int64_t* a_ptr, const int32_t* a_idx, const void* a_val, const void* c,
        const void* eta, double* S_out, double* bounds, void* base, hipStream_t s)
{
    const Layout o = layout(base, n, m);
    const unsigned pg = (unsigned)((std::max(n, m) + 255) / 256);
    hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(1), 0, s, o);
    hipLaunchKernelGGL(k_na_lam<T>, dim3(kLamBlocks), dim3(256), 0, s, L, (const T*)lam,
                       o.lam_part);
    hipLaunchKernelGGL(k_na_setup<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (const T*)r, (const T*)eta, a_ptr, a_idx, (const T*)a_val, m, o);
    hipLaunchKernelGGL(k_na_segments<T>, dim3(kSegBlocks), dim3(256), 0, s, L, n, seg_ptr, idx,
                       (const T*)v, (const T*)w, (const T*)v0, (const T*)lam, o);
    hipLaunchKernelGGL(k_na_fold<T>, dim3(pg), dim3(256), 0, s, n, m, (const T*)r, (const T*)c,
                       (const T*)eta, S_out, o);
    hipLaunchKernelGGL(k_na_final, dim3(1), dim3(256), 0, s, kSegBlocks, (int)pg, o, bounds);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CBLP_EHIP, std::string("cblp_gap_static: ") + hipGetErrorString(e));
    return CBLP_OK;
}

}  // namespace
}  // namespace cblp

using namespace cblp;

extern "C" int64_t cblp_gap_static_max_products(void) { return max_products(); }

extern "C" int cblp_gap_static(int64_t L, int64_t n, int64_t m, const int64_t* seg_ptr,
                               const int32_t* prod_idx, const void* v, const void* w,
                               const void* v0, const void* lambda, const void* r,
                               const int64_t* a_ptr, const int32_t* a_idx, const void* a_val,
                               const void* c, int32_t dtype, const void* eta, double* S_out,
                               double* bounds, void* stream)
{
    set_error(CBLP_OK, "");
    if (L < 0 || n <= 0 || m <= 0) return set_error(CBLP_EINVAL, "need L >= 0, n > 0, m > 0");
    if (n > max_products() || m > max_products())
        return set_error(CBLP_EINVAL, "cblp_gap_static: n and m must be at most " +
                                          std::to_string(max_products()) +
                                          " (the size of its static scratch)");
    if (dtype != CBLP_F32 && dtype != CBLP_F64) return set_error(CBLP_EINVAL, "bad dtype");
    const bool ident = !a_ptr && !a_idx && !a_val;
    if (!ident && (!a_ptr || !a_idx || !a_val))
        return set_error(CBLP_EINVAL, "a_ptr, a_idx, a_val must be all NULL or all set");
    if (ident && m != n) return set_error(CBLP_EINVAL, "identity resource matrix needs m == n");
    if (!seg_ptr || !r || !c || !eta || !bounds || (L > 0 && (!v0 || !lambda || !prod_idx || !v || !w)))
        return set_error(CBLP_EINVAL, "NULL argument");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return set_error(CBLP_EHIP, "hipGetDevice failed");
    void* base = nullptr;
    {
        // the device address of this GPU's copy of `scratch`, looked up once
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[dev]) {
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return set_error(CBLP_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                hipGetErrorString(e));
            g_scratch[dev] = ptr;
        }
        base = g_scratch[dev];
    }
    hipStream_t s = (hipStream_t)stream;
    return dtype == CBLP_F32
               ? run<float>(L, n, m, seg_ptr, prod_idx, v, w, v0, lambda, r, a_ptr, a_idx, a_val,
                            c, eta, S_out, bounds, base, s)
               : run<double>(L, n, m, seg_ptr, prod_idx, v, w, v0, lambda, r, a_ptr, a_idx,
                             a_val, c, eta, S_out, bounds, base, s);
}

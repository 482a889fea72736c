// Learned warm start for the capacity duals: per-product features, a small
// GELU MLP (4 -> 256 -> 256 -> 1) with BF16 weights and FP32 accumulation,
// trained on the GPU by its own forward and backward kernels, whose output
// eta_j = max(0, y_j) r_j starts spfom_solve.
//
// Features of product j (all from one pass over the library's sorted copy):
//   x0 = min(c_j / d_j, 4)    capacity over the demand when every segment is
//                             offered its whole set (nominal attractions),
//                             d_j = sum_l lambda_l v_lj / (v_l0 + sum_{N_l} v)
//                             (4 when d_j = 0)
//   x1 = r_j / max_k r_k
//   x2 = log1p((sum_l v_lj) n / L)      attraction mass, size-normalised
//   x3 = log1p(deg_j n / L)             number of segments considering j
// Sums are 64-bit fixed point (LDS bins for the head, atomics for the tail),
// so the features are bitwise reproducible.
//
// Rounding points (the CPU reference uses the same): the 256 x 256 layer's
// operands are BF16 (activations and W2, round to nearest even), the input
// and output layers use BF16-rounded weights with FP32 activations; every
// product accumulates in FP32; biases, GELU and the loss are FP32.
//
// The 256 x 256 products (forward Z2 = H1 W2, backward dW2 = H1^T dZ2 and
// dH1 = dZ2 W2^T) run on gfx950's v_mfma_f32_16x16x32_bf16.  A training step
// is two launches: k_train (forward, loss and backward of 64-row chunks per
// block, partial gradients per block) and k_train_reduce (the blocks' sum in
// a fixed order, Adam, the BF16 copies of W2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "common.hpp"
#include "handle.hpp"

namespace cblp {
namespace {

constexpr int IN = 4, HID = 256;
constexpr int64_t OFF_W1 = 0, OFF_B1 = OFF_W1 + IN * HID, OFF_W2 = OFF_B1 + HID,
                  OFF_B2 = OFF_W2 + HID * HID, OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID,
                  NPARAM = OFF_B3 + 1;
constexpr int kFeatBins = 2048;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float bfr(float x) { return bf2f(f2bf(x)); }

// GELU(z) = z Phi(z) and GELU'(z) = Phi(z) + z phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2,
// phi(z) = exp(-z^2 / 2) / sqrt(2 pi): one erf for both
__device__ __forceinline__ void gelu2(float z, float& g, float& d)
{
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    g = z * cdf;
    d = cdf + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}
__device__ __forceinline__ float gelu(float z)
{
    float g, d;
    gelu2(z, g, d);
    return g;
}

// ------------------------------------------------------------ features

template <typename T>
__global__ void k_feat_max(int64_t n, const T* r, int64_t nnz, const T* v, unsigned* mx)
{
    unsigned a = 0u, b = 0u;   // bit patterns of non-negative floats order like the values
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
        a = max(a, __float_as_uint(fmaxf((float)r[j], 0.0f)));
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += stride)
        b = max(b, __float_as_uint((float)v[q]));
    atomicMax(&mx[0], a);
    atomicMax(&mx[1], b);
}

struct FeatArgs {
    int64_t L, n;
    const int64_t* ptr;
    const int32_t* idx;
    const void* v;
    const void* v0;
    const void* lam;
    double dscale, ascale;         // fixed-point scales of demand and attraction mass
    int H;                         // LDS-binned products
    unsigned long long* part;      // [grid][3][H]: demand, attraction, degree
    unsigned long long* tail;      // [3][n] for products >= H
    const int32_t* pnew;           // [n] library id of caller product j; NULL: j
};

template <typename T>
__global__ void __launch_bounds__(256) k_feat_seg(FeatArgs a)
{
    __shared__ unsigned long long bd[kFeatBins], ba[kFeatBins], bg[kFeatBins];
    for (int j = threadIdx.x; j < a.H; j += blockDim.x) bd[j] = ba[j] = bg[j] = 0ull;
    __syncthreads();
    const T* v = (const T*)a.v;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.L;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = a.ptr[p], e = a.ptr[p + 1];
        double tot = (double)((const T*)a.v0)[p];
        for (int64_t q = b; q < e; ++q) tot += (double)v[q];
        const double f = (double)((const T*)a.lam)[p] / tot;
        for (int64_t q = b; q < e; ++q) {
            const int32_t j = a.idx[q];
            const double x = (double)v[q];
            const unsigned long long qd = (unsigned long long)__double2ll_rn(f * x * a.dscale);
            const unsigned long long qa = (unsigned long long)__double2ll_rn(x * a.ascale);
            if (j < a.H) {
                atomicAdd(&bd[j], qd);
                atomicAdd(&ba[j], qa);
                atomicAdd(&bg[j], 1ull);
            } else {
                atomicAdd(&a.tail[j], qd);
                atomicAdd(&a.tail[a.n + j], qa);
                atomicAdd(&a.tail[2 * a.n + j], 1ull);
            }
        }
    }
    __syncthreads();
    unsigned long long* out = a.part + (size_t)blockIdx.x * 3 * a.H;
    for (int j = threadIdx.x; j < a.H; j += blockDim.x) {
        out[j] = bd[j];
        out[a.H + j] = ba[j];
        out[2 * a.H + j] = bg[j];
    }
}

template <typename T>
__global__ void k_feat_fold(FeatArgs a, int nblocks, const T* r, const T* c, const unsigned* mx,
                            float* X)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const int64_t jq = a.pnew ? a.pnew[j] : j;   // the sorted copy's id of product j
    unsigned long long d = a.tail[jq], at = a.tail[a.n + jq], dg = a.tail[2 * a.n + jq];
    if (jq < a.H)
        for (int b = 0; b < nblocks; ++b) {
            const unsigned long long* pr = a.part + (size_t)b * 3 * a.H;
            d += pr[jq];
            at += pr[a.H + jq];
            dg += pr[2 * a.H + jq];
        }
    const double dem = (double)(long long)d / a.dscale;
    const double att = (double)(long long)at / a.ascale;
    const double rmax = (double)__uint_as_float(mx[0]);
    const double scale = a.L > 0 ? (double)a.n / (double)a.L : 0.0;
    const double cj = (double)c[j];
    float* x = X + j * IN;
    x[0] = (float)(dem > 0.0 ? fmin(cj / dem, 4.0) : 4.0);
    x[1] = (float)(rmax > 0.0 ? (double)r[j] / rmax : 0.0);
    x[2] = (float)log1p(att * scale);
    x[3] = (float)log1p((double)dg * scale);
}

// Per product (caller id j): demand, attraction mass and degree in FP64 from
// the fixed-point sums, for the resource features.
__global__ void k_feat_prod(FeatArgs a, int nblocks, double* prod3)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n) return;
    const int64_t jq = a.pnew ? a.pnew[j] : j;
    unsigned long long d = a.tail[jq], at = a.tail[a.n + jq], dg = a.tail[2 * a.n + jq];
    if (jq < a.H)
        for (int b = 0; b < nblocks; ++b) {
            const unsigned long long* pr = a.part + (size_t)b * 3 * a.H;
            d += pr[jq];
            at += pr[a.H + jq];
            dg += pr[2 * a.H + jq];
        }
    prod3[j] = (double)(long long)d / a.dscale;
    prod3[a.n + j] = (double)(long long)at / a.ascale;
    prod3[2 * a.n + j] = (double)dg;
}

// The scale of each resource's dual: the largest revenue per unit of the
// resource, max r_j / a_ij over its entries with a_ij > 0 (0 if none); the
// largest positive scale goes to *mx (non-negative doubles order like their
// bit patterns).
template <typename T>
__global__ void k_res_scale(int64_t m, const int64_t* at_ptr, const int32_t* at_prod,
                            const double* at_val, const T* r, double* scale,
                            unsigned long long* mx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double best = 0.0;
    bool any = false;
    for (int64_t q = at_ptr[i]; q < at_ptr[i + 1]; ++q) {
        const double w = at_val[q];
        if (!(w > 0.0)) continue;
        const double x = (double)r[at_prod[q]] / w;
        best = any ? fmax(best, x) : x;
        any = true;
    }
    scale[i] = best;
    if (mx) atomicMax(mx, (unsigned long long)__double_as_longlong(fmax(best, 0.0)));
}

// Features of resource i from the product sums weighted by its entries:
// capacity over sum_j a_ij d_j, scale over the largest scale, and the
// attraction mass and entry count of its products, size-normalised by m / L.
template <typename T>
__global__ void k_feat_res(int64_t m, int64_t L, const int64_t* at_ptr, const int32_t* at_prod,
                           const double* at_val, int64_t n, const double* prod3,
                           const double* scale, const unsigned long long* mx, const T* c, float* X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double D = 0.0, M = 0.0, G = 0.0;
    for (int64_t q = at_ptr[i]; q < at_ptr[i + 1]; ++q) {
        const int64_t j = at_prod[q];
        const double w = at_val[q];
        D += w * prod3[j];
        M += w * prod3[n + j];
        G += prod3[2 * n + j];
    }
    const double smax = __longlong_as_double((long long)*mx);
    const double sz = L > 0 ? (double)m / (double)L : 0.0;
    const double ci = (double)c[i];
    float* x = X + i * IN;
    x[0] = (float)(D > 0.0 ? fmin(ci / D, 4.0) : 4.0);
    x[1] = (float)(smax > 0.0 ? scale[i] / smax : 0.0);
    x[2] = (float)log1p(M * sz);
    x[3] = (float)log1p(G * sz);
}

// ------------------------------------------------------------ MLP layers

// MFMA operands: v_mfma_f32_16x16x32_bf16 (gfx950).  Lane l holds
// A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16], i = 0..7, and
// receives D[4 (l / 16) + i][l % 16], i = 0..3.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// eight consecutive BF16 values (16-byte aligned)
__device__ __forceinline__ v8bf ld8(const unsigned short* p)
{
    v8bf x;
    __builtin_memcpy(&x, p, 16);
    return x;
}

// eight BF16 values `stride` elements apart (LDS columns)
__device__ __forceinline__ v8bf ld8s(const unsigned short* p, int stride)
{
    unsigned short u[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) u[i] = p[i * stride];
    v8bf x;
    __builtin_memcpy(&x, u, 16);
    return x;
}

__device__ __forceinline__ v4f mfma32(v8bf a, v8bf b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// h1 = GELU(x W1 + b1) of kRows rows into LDS as BF16 (zero past `valid`
// rows); thread u computes hidden unit u.  z1 is formed as the backward pass
// re-forms it.
constexpr int kRows = 64;

__device__ __forceinline__ float z1_of(const float (*xs)[IN], int r, float b1, const float* w1)
{
    float z = b1;
#pragma unroll
    for (int k = 0; k < IN; ++k) z += xs[r][k] * w1[k];
    return z;
}

// Fused inference: y for 64 rows per block of four waves with no activation
// leaving the chip.  h1 is formed in LDS as BF16; each wave multiplies the
// four 16-row tiles by its 64 columns of W2 on the matrix cores, loading each
// B fragment once for the four tiles; then b2, GELU and the dot with BF16(w3)
// over its columns; the four waves' partial sums are added in wave order.
__global__ void __launch_bounds__(256) k_mlp_infer(const float* X, int64_t rows, const float* P,
                                                   const unsigned short* W2t, float* y)
{
    constexpr int RT = kRows / 16;
    __shared__ __attribute__((aligned(16))) unsigned short h1[kRows * HID];
    __shared__ float xs[kRows][IN];
    __shared__ float part[4][kRows];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * kRows;
    if (tid < kRows) {
        const int64_t row = m0 + tid;
#pragma unroll
        for (int k = 0; k < IN; ++k) xs[tid][k] = row < rows ? X[row * IN + k] : 0.0f;
    }
    __syncthreads();
    {
        const int u = tid;
        const float b1 = P[OFF_B1 + u];
        float w1[IN];
#pragma unroll
        for (int k = 0; k < IN; ++k) w1[k] = bfr(P[OFF_W1 + k * HID + u]);
        for (int r = 0; r < kRows; ++r)
            h1[r * HID + u] = f2bf(m0 + r < rows ? gelu(z1_of(xs, r, b1, w1)) : 0.0f);
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int n0 = wave * 64;
    const int r16 = lane & 15, g4 = lane >> 4;
    v4f acc[RT][4];
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m][t] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short* pb = W2t + (size_t)(n0 + r16) * HID + 8 * g4;
    for (int k0 = 0; k0 < HID; k0 += 32) {
        v8bf b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = ld8(pb + (size_t)16 * t * HID + k0);
#pragma unroll
        for (int m = 0; m < RT; ++m) {
            const v8bf a = ld8(h1 + (16 * m + r16) * HID + k0 + 8 * g4);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[m][t] = mfma32(a, b[t], acc[m][t]);
        }
    }
    float b2[4], w3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        b2[t] = P[OFF_B2 + n0 + 16 * t + r16];
        w3[t] = bfr(P[OFF_W3 + n0 + 16 * t + r16]);
    }
#pragma unroll
    for (int m = 0; m < RT; ++m) {
        float py[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // rows 16 m + 4 g4 + i, this lane's columns
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) py[i] += gelu(acc[m][t][i] + b2[t]) * w3[t];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            for (int o = 1; o < 16; o <<= 1) py[i] += __shfl_xor(py[i], o, 64);
        if (r16 == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) part[wave][16 * m + 4 * g4 + i] = py[i];
    }
    __syncthreads();
    if (tid < kRows && m0 + tid < rows)
        y[m0 + tid] = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + P[OFF_B3];
}

// One fused training pass (forward, mean-squared-error loss, backward) over
// the rows of a minibatch: rows r < cnt are (X, Y)[perm ? perm[r] : r].  A
// block of 16 waves takes chunks of kTRows rows (chunk c = block, block +
// grid, ...) and writes its partial gradient (the sum over its rows) to its
// own NPARAM slot of Gpart and its squared error to lpart, so k_train_reduce
// can add the blocks in a fixed order.  Per chunk:
//   h1 = GELU(z1), z1 = x W1 + b1             LDS, BF16 (and GELU'(z1), FP32)
//   Z2 = H1 W2                                matrix cores; wave w: columns 16w..
//   h2 = GELU(Z2 + b2), y = h2 . BF16(w3) + b3
//   dy = 2 (y - t) / cnt
//   dZ2 = dy BF16(w3) GELU'(Z2)               FP32 for the b2 sum, BF16 in LDS
//   dH1 = dZ2 W2^T                            matrix cores; wave w: units 16w..
//   dZ1 = dH1 GELU'(z1)
//   dW2 += H1^T dZ2                           matrix cores; wave w: rows 16w..
// and the column sums of h2 dy (w3), dy (b3), dZ2 (b2), dZ1 (b1), x_k dZ1
// (W1): thread (u, q) adds rows q, q + 4, ... of column u, and the four
// threads of a column are added in q order at the end.  GELU and its
// derivative share one erf per element.  The four waves of a SIMD hide each
// other's LDS and memory latency.
constexpr int kTRows = 32;
constexpr int kTThreads = 1024;
constexpr int64_t kGStride = (NPARAM + 3) / 4 * 4;   // partial slots on 16-byte boundaries

struct TrainArgs {
    const float* X;
    const float* Y;
    const int32_t* perm;
    int64_t cnt;
    float inv2;                    // 2 / cnt
    const float* P;
    const unsigned short* W2b;     // BF16 W2, [in][out]
    const unsigned short* W2t;     // BF16 W2 transposed, [out][in]
    float* Gpart;                  // [grid][kGStride]
    double* lpart;                 // [grid]
};

__global__ void __launch_bounds__(kTThreads) k_train(TrainArgs a)
{
    constexpr int RT = kTRows / 16;
    constexpr int RQ = kTThreads / HID;           // threads per column (4)
    constexpr int SEG = kTThreads / kTRows;       // column segments of the y sums (32)
    constexpr int SW = HID / SEG;                 // columns per segment (8)
    __shared__ __attribute__((aligned(16))) unsigned short h1[kTRows * HID];
    __shared__ __attribute__((aligned(16))) unsigned short dz[kTRows * HID];
    __shared__ float zs[kTRows * HID];    // z2 = Z2 + b2, then GELU'(z2)
    __shared__ float hs[kTRows * HID];    // h2, then dH1
    __shared__ float g1[kTRows * HID];    // GELU'(z1)
    __shared__ float xs[kTRows][IN];
    __shared__ float ys[kTRows];
    __shared__ float dys[kTRows];
    __shared__ double es[kTRows];         // squared errors
    __shared__ float w3s[HID];            // BF16(w3)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g4 = lane >> 4;
    float* G = a.Gpart + (size_t)blockIdx.x * kGStride;
    const int n0 = wave * 16;      // this wave's columns / hidden units / dW2 rows
    const int u = tid % HID, q = tid / HID;   // elementwise: column u, rows q, q + RQ, ...
    const float b1u = a.P[OFF_B1 + u], w3u = bfr(a.P[OFF_W3 + u]);
    const float b2w = a.P[OFF_B2 + n0 + r16];
    const float b3 = a.P[OFF_B3];
    float w1u[IN];
#pragma unroll
    for (int k = 0; k < IN; ++k) w1u[k] = bfr(a.P[OFF_W1 + k * HID + u]);
    if (tid < HID) w3s[tid] = w3u;
    float gw3 = 0.0f, gb2 = 0.0f, gb1 = 0.0f, gb3 = 0.0f;
    float gW1[IN] = {0.0f, 0.0f, 0.0f, 0.0f};
    double esum = 0.0;
    for (int64_t c = blockIdx.x; c * kTRows < a.cnt; c += gridDim.x) {
        const bool first = c == (int64_t)blockIdx.x;
        const int64_t m0 = c * kTRows;
        __syncthreads();           // the previous chunk is done with the LDS
        if (tid < kTRows) {
            const int64_t row = m0 + tid;
            if (row < a.cnt) {
                const int64_t qq = a.perm ? (int64_t)a.perm[row] : row;
#pragma unroll
                for (int k = 0; k < IN; ++k) xs[tid][k] = a.X[qq * IN + k];
                ys[tid] = a.Y[qq];
            } else {
#pragma unroll
                for (int k = 0; k < IN; ++k) xs[tid][k] = 0.0f;
                ys[tid] = 0.0f;
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int r = q; r < kTRows; r += RQ) {
            float g = 0.0f, d = 0.0f;
            if (m0 + r < a.cnt) gelu2(z1_of(xs, r, b1u, w1u), g, d);
            h1[r * HID + u] = f2bf(g);
            g1[r * HID + u] = d;
        }
        __syncthreads();
        // Z2 = H1 W2, plus b2, into zs
        {
            v4f acc[RT];
#pragma unroll
            for (int m = 0; m < RT; ++m) acc[m] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
            // the wave's eight W2 fragments in flight at once
            const unsigned short* pb = a.W2t + (size_t)(n0 + r16) * HID + 8 * g4;
            v8bf b[HID / 32];
#pragma unroll
            for (int kk = 0; kk < HID / 32; ++kk) b[kk] = ld8(pb + 32 * kk);
#pragma unroll
            for (int kk = 0; kk < HID / 32; ++kk)
#pragma unroll
                for (int m = 0; m < RT; ++m)
                    acc[m] = mfma32(ld8(h1 + (16 * m + r16) * HID + 32 * kk + 8 * g4), b[kk], acc[m]);
#pragma unroll
            for (int m = 0; m < RT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    zs[(16 * m + 4 * g4 + i) * HID + n0 + r16] = acc[m][i] + b2w;
        }
        __syncthreads();
        // h2 = GELU(z2) and GELU'(z2); y: thread (row, segment) sums its 8
        // columns, the 32 segments of a row (half a wave) are added by shuffles
        {
            const int row = tid / SEG, sg = tid % SEG;
            float py = 0.0f;
#pragma unroll
            for (int k = 0; k < SW; ++k) {
                const int o = row * HID + SW * sg + k;
                float g, d;
                gelu2(zs[o], g, d);
                hs[o] = g;
                zs[o] = d;
                py += g * w3s[SW * sg + k];
            }
#pragma unroll
            for (int o = 1; o < SEG; o <<= 1) py += __shfl_xor(py, o, 64);
            if (sg == 0) {
                float g = 0.0f;
                double e2 = 0.0;
                if (m0 + row < a.cnt) {
                    const float d = (py + b3) - ys[row];
                    g = d * a.inv2;
                    e2 = (double)d * (double)d;
                }
                dys[row] = g;
                es[row] = e2;
            }
        }
        __syncthreads();
        if (tid == 0)
            for (int r = 0; r < kTRows; ++r) {
                gb3 += dys[r];
                esum += es[r];
            }
        // dZ2 = dy BF16(w3) GELU'(z2) (BF16 into LDS); the w3 and b2 sums
#pragma unroll 2
        for (int r = q; r < kTRows; r += RQ) {
            const float dy = dys[r];
            const float g = dy * w3u * zs[r * HID + u];
            gw3 += hs[r * HID + u] * dy;
            gb2 += g;
            dz[r * HID + u] = f2bf(g);
        }
        __syncthreads();
        // dH1 = dZ2 W2^T into hs: B(n, k) = W2[k][n] = W2b[k HID + n]
        {
            v4f acc[RT];
#pragma unroll
            for (int m = 0; m < RT; ++m) acc[m] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
            const unsigned short* pw = a.W2b + (size_t)(n0 + r16) * HID + 8 * g4;
            v8bf b[HID / 32];
#pragma unroll
            for (int kk = 0; kk < HID / 32; ++kk) b[kk] = ld8(pw + 32 * kk);
#pragma unroll
            for (int kk = 0; kk < HID / 32; ++kk)
#pragma unroll
                for (int m = 0; m < RT; ++m)
                    acc[m] = mfma32(ld8(dz + (16 * m + r16) * HID + 32 * kk + 8 * g4), b[kk], acc[m]);
#pragma unroll
            for (int m = 0; m < RT; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) hs[(16 * m + 4 * g4 + i) * HID + n0 + r16] = acc[m][i];
        }
        // dW2 += H1^T dZ2 over the chunk's 32 rows, formed as its transpose
        // dZ2^T H1 (A(n, r) = dZ2[r][n], B(r, k) = h1[r][k]) so that each lane
        // holds four consecutive n of one row k of dW2: one 16-byte store
        {
            const v8bf bk = ld8s(h1 + (8 * g4) * HID + n0 + r16, HID);
            float* o = G + OFF_W2 + (size_t)(n0 + r16) * HID + 4 * g4;
#pragma unroll 2
            for (int nt = 0; nt < HID / 16; ++nt) {
                const v4f d = mfma32(ld8s(dz + (8 * g4) * HID + 16 * nt + r16, HID), bk,
                                     (v4f){0.0f, 0.0f, 0.0f, 0.0f});
                v4f* po = (v4f*)(o + 16 * nt);
                *po = first ? d : *po + d;
            }
        }
        __syncthreads();
        // dZ1 = dH1 GELU'(z1): the b1 and W1 sums
#pragma unroll 2
        for (int r = q; r < kTRows; r += RQ) {
            const float d1 = hs[r * HID + u] * g1[r * HID + u];
            gb1 += d1;
#pragma unroll
            for (int k = 0; k < IN; ++k) gW1[k] += xs[r][k] * d1;
        }
    }
    // the RQ threads of each column, added in q order
    __syncthreads();
    float* red = zs;               // [7][RQ][HID]
    red[(0 * RQ + q) * HID + u] = gw3;
    red[(1 * RQ + q) * HID + u] = gb2;
    red[(2 * RQ + q) * HID + u] = gb1;
#pragma unroll
    for (int k = 0; k < IN; ++k) red[((3 + k) * RQ + q) * HID + u] = gW1[k];
    __syncthreads();
    if (tid < HID) {
        float v[3 + IN];
#pragma unroll
        for (int x = 0; x < 3 + IN; ++x) {
            float t = red[(x * RQ) * HID + tid];
#pragma unroll
            for (int qq = 1; qq < RQ; ++qq) t += red[(x * RQ + qq) * HID + tid];
            v[x] = t;
        }
        G[OFF_W3 + tid] = v[0];
        G[OFF_B2 + tid] = v[1];
        G[OFF_B1 + tid] = v[2];
#pragma unroll
        for (int k = 0; k < IN; ++k) G[OFF_W1 + k * HID + tid] = v[3 + k];
    }
    if (tid == 0) {
        G[OFF_B3] = gb3;
        a.lpart[blockIdx.x] = esum;
    }
}

// The gradient: the nb block partials added in block order (FP64); with
// adam set, one Adam step (Kingma and Ba) on the FP32 master parameters and
// the BF16 copies of W2 re-rounded.  Thread i takes parameters 4i .. 4i + 3
// (16-byte loads, four blocks' loads in flight).  loss_acc (nullable) += the
// blocks' squared errors, added in block order by thread 0.
__global__ void __launch_bounds__(256) k_train_reduce(const float* Gpart, int nb,
                                                      const double* lpart, float* G, float* P,
                                                      float* M, float* V, int adam, float lr,
                                                      float b1, float b2, float eps, float c1,
                                                      float c2, unsigned short* W2b,
                                                      unsigned short* W2t, double* loss_acc)
{
    const int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i4 == 0 && loss_acc) {
        double e = 0.0;
        for (int b = 0; b < nb; ++b) e += lpart[b];
        loss_acc[0] += e;
    }
    if (4 * i4 >= NPARAM) return;
    constexpr int64_t S4 = kGStride / 4;
    const v4f* src = (const v4f*)Gpart + i4;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 4 <= nb; b += 4) {
        const v4f x0 = src[(size_t)b * S4], x1 = src[(size_t)(b + 1) * S4];
        const v4f x2 = src[(size_t)(b + 2) * S4], x3 = src[(size_t)(b + 3) * S4];
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = (((s[k] + (double)x0[k]) + (double)x1[k]) + (double)x2[k]) + (double)x3[k];
    }
    for (; b < nb; ++b) {
        const v4f x = src[(size_t)b * S4];
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += (double)x[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t i = 4 * i4 + k;
        if (i >= NPARAM) break;
        const float g = (float)s[k];
        G[i] = g;
        if (!adam) continue;
        const float m = b1 * M[i] + (1.0f - b1) * g;
        const float v = b2 * V[i] + (1.0f - b2) * g * g;
        M[i] = m;
        V[i] = v;
        const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
        P[i] = p;
        if (i >= OFF_W2 && i < OFF_W2 + HID * HID) {
            const int64_t q = i - OFF_W2;
            const unsigned short x = f2bf(p);
            W2b[q] = x;
            W2t[(q % HID) * HID + q / HID] = x;
        }
    }
}

// BF16 copies of W2 [256 x 256]: as stored (row i = input unit i) and transposed
__global__ void k_round_w2(const float* W2, unsigned short* out, unsigned short* outT)
{
    const int i = blockIdx.x, u = threadIdx.x;
    const unsigned short x = f2bf(W2[i * HID + u]);
    out[i * HID + u] = x;
    outT[u * HID + i] = x;
}

// eta_i = max(y_i, 0) scale_i (scale: r for A = I, the resource scale otherwise)
template <typename T, typename S>
__global__ void k_eta_from_y(const float* y, const S* r, int64_t n, T* eta)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) eta[j] = (T)(fmaxf(y[j], 0.0f) * (float)r[j]);
}

// y_i = eta_i / scale_i (0 where scale_i <= 0): the quantity the network predicts
template <typename T, typename S>
__global__ void k_targets(const T* eta, const S* r, int64_t n, float* Y)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) Y[j] = r[j] > (S)0 ? (float)((double)eta[j] / (double)r[j]) : 0.0f;
}

__global__ void k_fill_f64(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace
}  // namespace cblp

using namespace cblp;

struct wsnet {
    float* P = nullptr;            // FP32 master parameters [NPARAM]
    float* G = nullptr;            // gradients
    float* M = nullptr;            // Adam moments
    float* V = nullptr;
    unsigned short* W2b = nullptr; // BF16 copy of W2
    unsigned short* W2t = nullptr; // BF16 copy of W2 transposed
    int64_t step = 0;
    int64_t cap = 0;               // rows the prediction scratch holds
    float *X = nullptr, *y = nullptr;   // prediction: features and outputs
    int gcap = 0;                  // training blocks the partials hold
    float* Gpart = nullptr;        // [gcap][kGStride] per-block gradient partials
    double* lpart = nullptr;       // [gcap] per-block squared errors
    double* lacc = nullptr;        // loss accumulator
    double* pinned = nullptr;
};

namespace {

int mfail(int code, const std::string& m) { return set_error(code, m); }

#define MHIP(expr)                                                                     \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return mfail(CBLP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kTrainBlocks = 256;   // most blocks of one training pass

void net_free_scratch(wsnet* w)
{
    void* ptrs[] = {w->X, w->y, w->Gpart, w->lpart, w->lacc};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    w->X = w->y = w->Gpart = nullptr;
    w->lpart = w->lacc = nullptr;
    w->cap = 0;
    w->gcap = 0;
}

void net_release(wsnet* w)
{
    if (!w) return;
    net_free_scratch(w);
    void* ptrs[] = {w->P, w->G, w->M, w->V, w->W2b, w->W2t};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (w->pinned) (void)hipHostFree(w->pinned);
    delete w;
}

template <typename P>
int malloc_d(P** p, size_t bytes)
{
    *p = nullptr;
    if (hipMalloc((void**)p, bytes ? bytes : 8) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(CBLP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return CBLP_OK;
}

// prediction scratch for `rows` rows
int ensure_rows(wsnet* w, int64_t rows)
{
    const int64_t need = std::max<int64_t>(rows, 64);
    if (need <= w->cap) return CBLP_OK;
    if (w->X) (void)hipFree(w->X);
    if (w->y) (void)hipFree(w->y);
    w->X = w->y = nullptr;
    w->cap = 0;
    int rc;
    if ((rc = malloc_d(&w->X, (size_t)need * IN * 4)) || (rc = malloc_d(&w->y, (size_t)need * 4)))
        return rc;
    w->cap = need;
    return CBLP_OK;
}

int train_blocks(int64_t rows) { return (int)std::min<int64_t>(kTrainBlocks, (rows + kTRows - 1) / kTRows); }

// training partials for a pass over `rows` rows
int ensure_train(wsnet* w, int64_t rows)
{
    const int nb = train_blocks(rows);
    if (!w->lacc) {
        int rc;
        if ((rc = malloc_d(&w->lacc, 8))) return rc;
    }
    if (nb <= w->gcap) return CBLP_OK;
    if (w->Gpart) (void)hipFree(w->Gpart);
    if (w->lpart) (void)hipFree(w->lpart);
    w->Gpart = nullptr;
    w->lpart = nullptr;
    w->gcap = 0;
    int rc;
    if ((rc = malloc_d(&w->Gpart, (size_t)nb * kGStride * 4)) || (rc = malloc_d(&w->lpart, (size_t)nb * 8)))
        return rc;
    w->gcap = nb;
    return CBLP_OK;
}

// one training pass over rows (X, Y)[perm ? perm[r] : r], r < rows: the
// gradient into w->G, the squared error added to w->lacc, and with lr > 0 an
// Adam step.  Two launches.
int train_pass(wsnet* w, const float* X, const float* Y, const int32_t* perm, int64_t rows, float lr,
               hipStream_t s)
{
    const int nb = train_blocks(rows);
    TrainArgs a;
    a.X = X;
    a.Y = Y;
    a.perm = perm;
    a.cnt = rows;
    a.inv2 = 2.0f / (float)rows;
    a.P = w->P;
    a.W2b = w->W2b;
    a.W2t = w->W2t;
    a.Gpart = w->Gpart;
    a.lpart = w->lpart;
    hipLaunchKernelGGL(k_train, dim3(nb), dim3(kTThreads), 0, s, a);
    float c1 = 1.0f, c2 = 1.0f;
    const float b1 = 0.9f, b2 = 0.999f;
    if (lr > 0.0f) {
        w->step += 1;
        c1 = 1.0f - std::pow(b1, (float)w->step);
        c2 = 1.0f - std::pow(b2, (float)w->step);
    }
    hipLaunchKernelGGL(k_train_reduce, dim3((unsigned)((NPARAM + 1023) / 1024)), dim3(256), 0, s,
                       w->Gpart, nb, w->lpart, w->G, w->P, w->M, w->V, lr > 0.0f ? 1 : 0, lr, b1, b2,
                       1e-8f, c1, c2, w->W2b, w->W2t, w->lacc);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

// the loss accumulator: cleared / read back (synchronises)
int loss_clear(wsnet* w, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, w->lacc, (int64_t)1, 0.0);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

int loss_read(wsnet* w, double* out, hipStream_t s)
{
    MHIP(hipMemcpyAsync(w->pinned, w->lacc, 8, hipMemcpyDeviceToHost, s));
    MHIP(hipStreamSynchronize(s));
    *out = w->pinned[0];
    return CBLP_OK;
}

template <typename T>
int features_impl(cblp_instance* h, float* X, hipStream_t s)
{
    unsigned* mx = nullptr;
    int rc;
    if ((rc = malloc_d(&mx, 8))) return rc;
    std::vector<unsigned> hm(2, 0u);
    hipError_t e = hipMemsetAsync(mx, 0, 8, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_feat_max<T>, dim3(1024), dim3(256), 0, s, h->n, (const T*)h->r, h->nnz,
                           (const T*)h->v2, mx);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hm.data(), mx, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(mx);
        return mfail(CBLP_EHIP, std::string("feature bounds: ") + hipGetErrorString(e));
    }
    float vmax;
    std::memcpy(&vmax, &hm[1], 4);
    FeatArgs a;
    a.L = h->L;
    a.n = h->n;
    a.ptr = h->ptr2;
    a.idx = h->idx2;
    a.pnew = h->pnew;
    a.v = h->v2;
    a.v0 = h->v0c;
    a.lam = h->lam2;
    a.dscale = h->fx_scale;
    int ex = 0;
    std::frexp((double)vmax * (double)std::max<int64_t>(h->nnz, 1) + 1.0, &ex);
    a.ascale = std::ldexp(1.0, std::min(40, 61 - ex));
    a.H = (int)std::min<int64_t>(h->n, kFeatBins);
    const int grid = 1024;
    unsigned long long *part = nullptr, *tail = nullptr;
    if ((rc = malloc_d(&part, (size_t)grid * 3 * a.H * 8)) ||
        (rc = malloc_d(&tail, (size_t)3 * h->n * 8))) {
        (void)hipFree(mx);
        if (part) (void)hipFree(part);
        return rc;
    }
    a.part = part;
    a.tail = tail;
    // a resource matrix: product sums, resource scales and their largest
    double *prod3 = nullptr, *scale = nullptr;
    unsigned long long* smax = nullptr;
    if (h->a_ptr && ((rc = malloc_d(&prod3, (size_t)3 * h->n * 8)) ||
                     (rc = malloc_d(&scale, (size_t)h->m * 8)) || (rc = malloc_d(&smax, 8)))) {
        void* ptrs[] = {mx, part, tail, prod3, scale};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
        return rc;
    }
    e = hipMemsetAsync(tail, 0, (size_t)3 * h->n * 8, s);
    if (e == hipSuccess && smax) e = hipMemsetAsync(smax, 0, 8, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_feat_seg<T>, dim3(grid), dim3(256), 0, s, a);
        if (!h->a_ptr) {
            hipLaunchKernelGGL(k_feat_fold<T>, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0, s,
                               a, grid, (const T*)h->r, (const T*)h->c, mx, X);
        } else {
            const unsigned gm = (unsigned)((h->m + 255) / 256);
            hipLaunchKernelGGL(k_feat_prod, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0, s, a,
                               grid, prod3);
            hipLaunchKernelGGL(k_res_scale<T>, dim3(gm), dim3(256), 0, s, h->m, h->at_ptr,
                               h->at_prod, h->at_val, (const T*)h->r, scale, smax);
            hipLaunchKernelGGL(k_feat_res<T>, dim3(gm), dim3(256), 0, s, h->m, h->L, h->at_ptr,
                               h->at_prod, h->at_val, h->n, prod3, scale, smax,
                               (const T*)h->c, X);
        }
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    void* ptrs[] = {mx, part, tail, prod3, scale, smax};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (e != hipSuccess) return mfail(CBLP_EHIP, std::string("features: ") + hipGetErrorString(e));
    return CBLP_OK;
}

// the scale of every dual of h (resource matrix) into a fresh device array
// the caller frees
template <typename T>
int res_scale(cblp_instance* h, double** out, hipStream_t s)
{
    int rc;
    if ((rc = malloc_d(out, (size_t)h->m * 8))) return rc;
    hipLaunchKernelGGL(k_res_scale<T>, dim3((unsigned)((h->m + 255) / 256)), dim3(256), 0, s, h->m,
                       h->at_ptr, h->at_prod, h->at_val, (const T*)h->r, *out,
                       (unsigned long long*)nullptr);
    if (hipGetLastError() != hipSuccess) {
        (void)hipFree(*out);
        *out = nullptr;
        return mfail(CBLP_EHIP, "resource scale kernel failed");
    }
    return CBLP_OK;
}

}  // namespace

extern "C" {

int64_t wsnet_num_params(void) { return NPARAM; }

int wsnet_create(wsnet_t* out, uint64_t seed, void* stream)
{
    set_error(CBLP_OK, "");
    if (!out) return mfail(CBLP_EINVAL, "out is NULL");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    wsnet* w = new (std::nothrow) wsnet();
    if (!w) return mfail(CBLP_ENOMEM, "host allocation failed");
    int rc;
    if ((rc = malloc_d(&w->P, NPARAM * 4)) || (rc = malloc_d(&w->G, NPARAM * 4)) ||
        (rc = malloc_d(&w->M, NPARAM * 4)) || (rc = malloc_d(&w->V, NPARAM * 4)) ||
        (rc = malloc_d(&w->W2b, (size_t)HID * HID * 2)) ||
        (rc = malloc_d(&w->W2t, (size_t)HID * HID * 2))) {
        net_release(w);
        return rc;
    }
    if (hipHostMalloc((void**)&w->pinned, 16, hipHostMallocDefault) != hipSuccess) {
        net_release(w);
        return mfail(CBLP_ENOMEM, "hipHostMalloc failed");
    }
    // He-normal weights (GELU layers), zero biases, small output layer
    std::vector<float> p(NPARAM, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.0f, 1.0f);
    for (int64_t i = 0; i < IN * HID; ++i) p[OFF_W1 + i] = nd(rng) * std::sqrt(2.0f / IN);
    for (int64_t i = 0; i < HID * HID; ++i) p[OFF_W2 + i] = nd(rng) * std::sqrt(2.0f / HID);
    for (int64_t i = 0; i < HID; ++i) p[OFF_W3 + i] = nd(rng) * std::sqrt(1.0f / HID);
    if (hipMemcpyAsync(w->P, p.data(), NPARAM * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(w->M, 0, NPARAM * 4, s) != hipSuccess ||
        hipMemsetAsync(w->V, 0, NPARAM * 4, s) != hipSuccess ||
        hipMemsetAsync(w->G, 0, NPARAM * 4, s) != hipSuccess) {
        net_release(w);
        return mfail(CBLP_EHIP, "initialising the network failed");
    }
    hipLaunchKernelGGL(k_round_w2, dim3(HID), dim3(HID), 0, s, w->P + OFF_W2, w->W2b, w->W2t);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        net_release(w);
        return mfail(CBLP_EHIP, "initialising the network failed");
    }
    *out = w;
    return CBLP_OK;
}

void wsnet_destroy(wsnet_t w) { net_release(w); }

int wsnet_params(wsnet_t w, float* get, const float* set, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w) return mfail(CBLP_EINVAL, "net is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (set) {
        MHIP(hipMemcpyAsync(w->P, set, NPARAM * 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_round_w2, dim3(HID), dim3(HID), 0, s, w->P + OFF_W2, w->W2b, w->W2t);
        MHIP(hipGetLastError());
        w->step = 0;
        MHIP(hipMemsetAsync(w->M, 0, NPARAM * 4, s));
        MHIP(hipMemsetAsync(w->V, 0, NPARAM * 4, s));
    }
    if (get) MHIP(hipMemcpyAsync(get, w->P, NPARAM * 4, hipMemcpyDeviceToHost, s));
    MHIP(hipStreamSynchronize(s));
    return CBLP_OK;
}

int wsnet_features(cblp_t h, float* X, void* stream)
{
    set_error(CBLP_OK, "");
    if (!h || !X) return mfail(CBLP_EINVAL, "NULL handle or X");
    hipStream_t s = (hipStream_t)stream;
    return h->dtype == CBLP_F32 ? features_impl<float>(h, X, s) : features_impl<double>(h, X, s);
}

int wsnet_forward(wsnet_t w, const float* X, int64_t rows, float* y, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !X || !y || rows < 0) return mfail(CBLP_EINVAL, "NULL argument or rows < 0");
    if (rows == 0) return CBLP_OK;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((rows + kRows - 1) / kRows)),
                       dim3(256), 0, s, X, rows,
                       w->P, w->W2t, y);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

int wsnet_gradients(wsnet_t w, const float* X, const float* Y, int64_t rows, float* grads,
                    double* loss, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !X || !Y || rows < 1) return mfail(CBLP_EINVAL, "NULL argument or rows < 1");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ensure_train(w, rows)) || (rc = loss_clear(w, s)) ||
        (rc = train_pass(w, X, Y, nullptr, rows, 0.0f, s)))
        return rc;
    if (grads) MHIP(hipMemcpyAsync(grads, w->G, NPARAM * 4, hipMemcpyDeviceToDevice, s));
    double e = 0.0;
    if ((rc = loss_read(w, &e, s))) return rc;
    if (loss) *loss = e / (double)rows;
    return CBLP_OK;
}

int wsnet_train_step(wsnet_t w, const float* X, const float* Y, int64_t rows, float lr,
                     double* loss, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !X || !Y || rows < 1 || !(lr > 0.0f)) return mfail(CBLP_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ensure_train(w, rows))) return rc;
    if (loss && (rc = loss_clear(w, s))) return rc;
    if ((rc = train_pass(w, X, Y, nullptr, rows, lr, s))) return rc;
    if (loss) {
        double e = 0.0;
        if ((rc = loss_read(w, &e, s))) return rc;
        *loss = e / (double)rows;
    }
    return CBLP_OK;
}

int wsnet_train_epochs(wsnet_t w, const float* X, const float* Y, int64_t rows, int64_t batch,
                       int32_t epochs, float lr, uint64_t seed, double* losses, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !X || !Y || rows < 1 || batch < 1 || epochs < 0 || !(lr > 0.0f))
        return mfail(CBLP_EINVAL, "bad argument");
    if (rows > INT32_MAX) return mfail(CBLP_EINVAL, "rows above 2^31 - 1");
    hipStream_t s = (hipStream_t)stream;
    batch = std::min(batch, rows);
    int rc;
    if ((rc = ensure_train(w, batch))) return rc;
    int32_t* perm = nullptr;
    if ((rc = malloc_d(&perm, (size_t)rows * 4))) return rc;
    std::vector<int32_t> hp(rows);
    std::mt19937_64 rng(seed);
    for (int32_t e = 0; e < epochs && rc == CBLP_OK; ++e) {
        for (int64_t i = 0; i < rows; ++i) hp[i] = (int32_t)i;
        for (int64_t i = rows - 1; i > 0; --i) {        // Fisher-Yates
            const int64_t k = (int64_t)(rng() % (uint64_t)(i + 1));
            std::swap(hp[i], hp[k]);
        }
        if (hipMemcpyAsync(perm, hp.data(), (size_t)rows * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = mfail(CBLP_EHIP, "uploading the minibatch order failed");
            break;
        }
        if ((rc = loss_clear(w, s))) break;
        // each minibatch's mean loss weighted by its rows: the accumulator gets
        // the sum of squared errors
        for (int64_t b0 = 0; b0 < rows && rc == CBLP_OK; b0 += batch)
            rc = train_pass(w, X, Y, perm + b0, std::min(batch, rows - b0), lr, s);
        if (rc) break;
        double h = 0.0;
        if ((rc = loss_read(w, &h, s))) break;
        if (losses) losses[e] = h / (double)rows;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(perm);
    return rc;
}

int wsnet_targets(cblp_t h, const void* eta, float* Y, void* stream)
{
    set_error(CBLP_OK, "");
    if (!h || !eta || !Y) return mfail(CBLP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = (unsigned)((h->m + 255) / 256);
    if (!h->a_ptr) {
        if (h->dtype == CBLP_F32)
            hipLaunchKernelGGL((k_targets<float, float>), dim3(g), dim3(256), 0, s, (const float*)eta,
                               (const float*)h->r, h->m, Y);
        else
            hipLaunchKernelGGL((k_targets<double, double>), dim3(g), dim3(256), 0, s,
                               (const double*)eta, (const double*)h->r, h->m, Y);
        MHIP(hipGetLastError());
        return CBLP_OK;
    }
    double* scale = nullptr;
    int rc = h->dtype == CBLP_F32 ? res_scale<float>(h, &scale, s) : res_scale<double>(h, &scale, s);
    if (rc) return rc;
    if (h->dtype == CBLP_F32)
        hipLaunchKernelGGL((k_targets<float, double>), dim3(g), dim3(256), 0, s, (const float*)eta,
                           scale, h->m, Y);
    else
        hipLaunchKernelGGL((k_targets<double, double>), dim3(g), dim3(256), 0, s, (const double*)eta,
                           scale, h->m, Y);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(scale);
    if (e1 != hipSuccess || e2 != hipSuccess) return mfail(CBLP_EHIP, "targets kernel failed");
    return CBLP_OK;
}

int wsnet_predict(wsnet_t w, cblp_t h, void* eta, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !h || !eta) return mfail(CBLP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ensure_rows(w, h->m))) return rc;
    rc = h->dtype == CBLP_F32 ? features_impl<float>(h, w->X, s) : features_impl<double>(h, w->X, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((h->m + kRows - 1) / kRows)),
                       dim3(256), 0, s, w->X, h->m,
                       w->P, w->W2t, w->y);
    const unsigned g = (unsigned)((h->m + 255) / 256);
    if (!h->a_ptr) {
        if (h->dtype == CBLP_F32)
            hipLaunchKernelGGL((k_eta_from_y<float, float>), dim3(g), dim3(256), 0, s, w->y,
                               (const float*)h->r, h->m, (float*)eta);
        else
            hipLaunchKernelGGL((k_eta_from_y<double, double>), dim3(g), dim3(256), 0, s, w->y,
                               (const double*)h->r, h->m, (double*)eta);
        MHIP(hipGetLastError());
        return CBLP_OK;
    }
    double* scale = nullptr;
    rc = h->dtype == CBLP_F32 ? res_scale<float>(h, &scale, s) : res_scale<double>(h, &scale, s);
    if (rc) return rc;
    if (h->dtype == CBLP_F32)
        hipLaunchKernelGGL((k_eta_from_y<float, double>), dim3(g), dim3(256), 0, s, w->y, scale,
                           h->m, (float*)eta);
    else
        hipLaunchKernelGGL((k_eta_from_y<double, double>), dim3(g), dim3(256), 0, s, w->y, scale,
                           h->m, (double*)eta);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(scale);
    if (e1 != hipSuccess || e2 != hipSuccess) return mfail(CBLP_EHIP, "prediction kernels failed");
    return CBLP_OK;
}

int wsnet_start(wsnet_t w, cblp_t h, void* eta, int32_t* used, double* d_pred, double* d_zero,
                void* stream)
{
    int rc = wsnet_predict(w, h, eta, stream);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    spfom_stats st;
    if ((rc = cblp_gap(h, eta, &st, stream))) return rc;
    const double dp = st.trace[SPFOM_TR_DUAL];
    void* zeros = nullptr;
    const size_t bytes = (size_t)h->m * h->esz;
    if (hipMalloc(&zeros, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return mfail(CBLP_ENOMEM, "no memory for the cold-start duals");
    }
    if (hipMemsetAsync(zeros, 0, bytes, s) != hipSuccess) {
        (void)hipFree(zeros);
        return mfail(CBLP_EHIP, "clearing the cold-start duals failed");
    }
    rc = cblp_gap(h, zeros, &st, stream);
    (void)hipFree(zeros);
    if (rc) return rc;
    const double d0 = st.trace[SPFOM_TR_DUAL];
    // both are upper bounds on the LP optimum: keep the prediction only if its
    // bound is the tighter one
    const bool keep = dp < d0;
    if (!keep) {
        MHIP(hipMemsetAsync(eta, 0, bytes, s));
        MHIP(hipStreamSynchronize(s));
    }
    if (used) *used = keep ? 1 : 0;
    if (d_pred) *d_pred = dp;
    if (d_zero) *d_zero = d0;
    return CBLP_OK;
}

}  // extern "C"

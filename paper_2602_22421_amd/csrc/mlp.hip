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
// dH1 = dZ2 W2^T) run on v_mfma_f32_16x16x16_bf16: each wave owns a 16 x 16
// output tile; lane l holds A[l % 16][4 (l / 16) + i], B[4 (l / 16) + i][l % 16]
// and D[4 (l / 16) + i][l % 16], i = 0..3.
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
constexpr int kColRows = 256;     // rows per column-sum block

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

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * 0.39894228040143268f * expf(-0.5f * x * x);
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

// ------------------------------------------------------------ MLP layers

// z1 = X W1 + b1, h1 = GELU(z1) stored as BF16; rows past `rows` are zero
__global__ void __launch_bounds__(HID) k_l1_fwd(const float* X, int64_t rows, const float* P,
                                                float* z1, unsigned short* h1b)
{
    const int64_t r = blockIdx.x;
    const int u = threadIdx.x;
    float z = 0.0f;
    if (r < rows) {
        z = P[OFF_B1 + u];
        for (int k = 0; k < IN; ++k) z += X[r * IN + k] * bfr(P[OFF_W1 + k * HID + u]);
    }
    z1[r * HID + u] = z;
    h1b[r * HID + u] = f2bf(r < rows ? gelu(z) : 0.0f);
}

// C(m, n) = sum_k A(m, k) B(k, n), BF16 operands, FP32 accumulation.
// A(m, k) = TA ? A[k lda + m] : A[m lda + k];  B(k, n) = TB ? B[n ldb + k] : B[k ldb + n].
// EPI 0 stores C; EPI 1 stores z = C + bias[n] and h = GELU(z).
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm(const unsigned short* A, const unsigned short* B,
                                              float* C, int N, int K, int lda, int ldb,
                                              const float* bias, float* hout)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 64 + wave * 16;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = k0 + kq + i;
            a[i] = (short)(TA ? A[(size_t)k * lda + m0 + r] : A[(size_t)(m0 + r) * lda + k]);
            b[i] = (short)(TB ? B[(size_t)(n0 + r) * ldb + k] : B[(size_t)k * ldb + n0 + r]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const size_t o = (size_t)(m0 + kq + i) * N + n0 + r;
        if (EPI == 0) {
            C[o] = acc[i];
        } else {
            const float z = acc[i] + bias[n0 + r];
            C[o] = z;
            hout[o] = gelu(z);
        }
    }
}

// Row-block product for operands whose k index is contiguous in memory:
// C(m, n) = sum_k A[m lda + k] Bt[n ldb + k] over all N = 256 columns.  A
// block of four waves owns 16 rows; each wave owns 64 columns (four 16 x 16
// tiles) and reuses its A fragment, one 8-byte load per k step, for the four
// products.  EPI as k_gemm.
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_rows(const unsigned short* A, const unsigned short* Bt,
                                                   float* C, int N, int K, int lda, int ldb,
                                                   const float* bias, float* hout)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * 16, n0 = wave * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4f acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short* pa = A + (size_t)(m0 + r) * lda + kq;
    const unsigned short* pb = Bt + (size_t)(n0 + r) * ldb + kq;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const v4s a = *(const v4s*)(pa + k0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4s b = *(const v4s*)(pb + (size_t)16 * t * ldb + k0);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = n0 + 16 * t + r;
            const size_t o = (size_t)(m0 + kq + i) * N + n;
            if (EPI == 0) {
                C[o] = acc[t][i];
            } else {
                const float z = acc[t][i] + bias[n];
                C[o] = z;
                hout[o] = gelu(z);
            }
        }
}

// Fused inference: y for 64 rows per block of four waves with no activation
// leaving the chip.  h1 = GELU(x W1 + b1) is formed in LDS as BF16 (same
// operations as k_l1_fwd); each wave multiplies the four 16-row tiles by its
// 64 columns of W2 on the matrix cores, loading each B fragment once for the
// four tiles; then b2, GELU and the dot with BF16(w3) over its columns; the
// four waves' partial sums are added in wave order.
constexpr int kInferRows = 64;

__global__ void __launch_bounds__(256) k_mlp_infer(const float* X, int64_t rows, const float* P,
                                                   const unsigned short* W2t, float* y)
{
    constexpr int RT = kInferRows / 16;
    __shared__ __attribute__((aligned(16))) unsigned short h1[kInferRows * HID];
    __shared__ float part[4][kInferRows];
    const int tid = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * kInferRows;
    {
        const int u = tid;
        const float b1 = P[OFF_B1 + u];
        float w1[IN];
#pragma unroll
        for (int k = 0; k < IN; ++k) w1[k] = bfr(P[OFF_W1 + k * HID + u]);
        for (int r = 0; r < kInferRows; ++r) {
            const int64_t row = m0 + r;
            float v = 0.0f;
            if (row < rows) {
                float z = b1;
#pragma unroll
                for (int k = 0; k < IN; ++k) z += X[row * IN + k] * w1[k];
                v = gelu(z);
            }
            h1[r * HID + u] = f2bf(v);
        }
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int n0 = wave * 64;
    const int r = lane & 15, kq = (lane >> 4) * 4;
    v4f acc[RT][4];
#pragma unroll
    for (int m = 0; m < RT; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m][t] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
    const unsigned short* pb = W2t + (size_t)(n0 + r) * HID + kq;
    for (int k0 = 0; k0 < HID; k0 += 16) {
        v4s bfr4[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) bfr4[t] = *(const v4s*)(pb + (size_t)16 * t * HID + k0);
#pragma unroll
        for (int m = 0; m < RT; ++m) {
            const v4s a = *(const v4s*)(h1 + (16 * m + r) * HID + k0 + kq);
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bfr4[t], acc[m][t], 0, 0, 0);
        }
    }
    float b2[4], w3[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        b2[t] = P[OFF_B2 + n0 + 16 * t + r];
        w3[t] = bfr(P[OFF_W3 + n0 + 16 * t + r]);
    }
#pragma unroll
    for (int m = 0; m < RT; ++m) {
        float py[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // rows 16 m + kq + i, this lane's columns
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) py[i] += gelu(acc[m][t][i] + b2[t]) * w3[t];
        // sum over the 16 lanes of each row group (same kq)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            for (int o = 1; o < 16; o <<= 1) py[i] += __shfl_xor(py[i], o, 64);
        if (r == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) part[wave][16 * m + kq + i] = py[i];
    }
    __syncthreads();
    if (tid < kInferRows && m0 + tid < rows)
        y[m0 + tid] = ((part[0][tid] + part[1][tid]) + (part[2][tid] + part[3][tid])) + P[OFF_B3];
}

// y = h2 . w3 + b3, one wave per row
__global__ void __launch_bounds__(256) k_l3_fwd(const float* h2, const float* P, int64_t rpad,
                                                float* y)
{
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rpad) return;
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) s += h2[r * HID + lane * 4 + i] * bfr(P[OFF_W3 + lane * 4 + i]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) y[r] = s + P[OFF_B3];
}

// dy = 2 (y - t) / rows on real rows, 0 on padding; per-block squared error
__global__ void __launch_bounds__(256) k_dy(const float* y, const float* t, int64_t rows,
                                            int64_t rpad, float* dy, double* lpart)
{
    __shared__ double sh[256];
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    if (r < rpad) {
        float g = 0.0f;
        if (r < rows) {
            const float d = y[r] - t[r];
            g = 2.0f * d / (float)rows;
            e2 = (double)d * (double)d;
        }
        dy[r] = g;
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

// dz2 = dy w3 GELU'(z2), kept in FP32 and BF16
__global__ void __launch_bounds__(HID) k_l3_bwd(const float* dy, const float* z2, const float* P,
                                                float* dz2, unsigned short* dz2b)
{
    const int64_t r = blockIdx.x;
    const int u = threadIdx.x;
    const float g = dy[r] * bfr(P[OFF_W3 + u]) * gelu_d(z2[r * HID + u]);
    dz2[r * HID + u] = g;
    dz2b[r * HID + u] = f2bf(g);
}

// dz1 = dh1 GELU'(z1)
__global__ void __launch_bounds__(HID) k_l1_bwd(const float* dh1, const float* z1, float* dz1)
{
    const int64_t o = (int64_t)blockIdx.x * HID + threadIdx.x;
    dz1[o] = dh1[o] * gelu_d(z1[o]);
}

// out[u] = sum_r M[r ld + u] (s ? s[r sst] : 1) over rows [0, rpad): blocks of
// kColRows rows write FP64 partials; k_colsum_final adds them in block order.
__global__ void k_colsum(const float* M, int64_t ld, int64_t rpad, int ncols, const float* s,
                         int64_t sst, double* part)
{
    const int u = threadIdx.x;
    if (u >= ncols) return;
    const int64_t r0 = (int64_t)blockIdx.x * kColRows;
    const int64_t r1 = min(rpad, r0 + (int64_t)kColRows);
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc += (double)M[r * ld + u] * (s ? (double)s[r * sst] : 1.0);
    part[(size_t)blockIdx.x * ncols + u] = acc;
}

__global__ void k_colsum_final(const double* part, int nb, int ncols, float* out)
{
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ncols) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) acc += part[(size_t)b * ncols + u];
    out[u] = (float)acc;
}

__global__ void k_adam(float* P, const float* G, float* M, float* V, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = G[i];
    const float m = b1 * M[i] + (1.0f - b1) * g;
    const float v = b2 * V[i] + (1.0f - b2) * g * g;
    M[i] = m;
    V[i] = v;
    P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// BF16 copies of W2 [256 x 256]: as stored (row i = input unit i) and transposed
__global__ void k_round_w2(const float* W2, unsigned short* out, unsigned short* outT)
{
    const int i = blockIdx.x, u = threadIdx.x;
    const unsigned short x = f2bf(W2[i * HID + u]);
    out[i * HID + u] = x;
    outT[u * HID + i] = x;
}

template <typename T>
__global__ void k_eta_from_y(const float* y, const T* r, int64_t n, T* eta)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) eta[j] = (T)(fmaxf(y[j], 0.0f) * (float)r[j]);
}

// y_j = eta_j / r_j (0 where r_j <= 0): the quantity the network predicts
template <typename T>
__global__ void k_targets(const T* eta, const T* r, int64_t n, float* Y)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) Y[j] = r[j] > (T)0 ? (float)((double)eta[j] / (double)r[j]) : 0.0f;
}

// minibatch rows perm[0..cnt) of (X, Y) into (Xb, Yb), zero padding up to rpad
__global__ void k_gather(const float* X, const float* Y, const int32_t* perm, int64_t cnt,
                         int64_t rpad, float* Xb, float* Yb)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rpad) return;
    if (r < cnt) {
        const int64_t q = perm[r];
#pragma unroll
        for (int k = 0; k < IN; ++k) Xb[r * IN + k] = X[q * IN + k];
        Yb[r] = Y[q];
    } else {
#pragma unroll
        for (int k = 0; k < IN; ++k) Xb[r * IN + k] = 0.0f;
        Yb[r] = 0.0f;
    }
}

// acc[0] += sum of the nb loss partials (one thread, fixed order)
__global__ void k_loss_add(const double* part, int nb, double* acc)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0;
    for (int b = 0; b < nb; ++b) a += part[b];
    acc[0] += a;
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
    int64_t cap = 0;               // padded rows the scratch holds
    float *z1 = nullptr, *z2 = nullptr, *h2 = nullptr, *y = nullptr, *dy = nullptr;
    float *dz2 = nullptr, *dh1 = nullptr, *dz1 = nullptr, *X = nullptr, *Yb = nullptr;
    unsigned short *h1b = nullptr, *dz2b = nullptr;
    double* part = nullptr;        // column-sum partials
    double* lpart = nullptr;       // loss partials
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

void net_free_scratch(wsnet* w)
{
    void* ptrs[] = {w->z1, w->z2, w->h2, w->y, w->dy, w->dz2, w->dh1, w->dz1, w->X, w->Yb,
                    w->h1b, w->dz2b, w->part, w->lpart};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    w->z1 = w->z2 = w->h2 = w->y = w->dy = w->dz2 = w->dh1 = w->dz1 = w->X = w->Yb = nullptr;
    w->h1b = w->dz2b = nullptr;
    w->part = w->lpart = nullptr;
    w->cap = 0;
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

int64_t pad16(int64_t x) { return (x + 15) / 16 * 16; }

int ensure_scratch(wsnet* w, int64_t rows)
{
    const int64_t need = pad16(std::max<int64_t>(rows, 16));
    if (need <= w->cap) return CBLP_OK;
    net_free_scratch(w);
    const size_t a = (size_t)need * HID;
    int rc;
    if ((rc = malloc_d(&w->z1, a * 4)) || (rc = malloc_d(&w->z2, a * 4)) ||
        (rc = malloc_d(&w->h2, a * 4)) || (rc = malloc_d(&w->dz2, a * 4)) ||
        (rc = malloc_d(&w->dh1, a * 4)) || (rc = malloc_d(&w->dz1, a * 4)) ||
        (rc = malloc_d(&w->h1b, a * 2)) || (rc = malloc_d(&w->dz2b, a * 2)) ||
        (rc = malloc_d(&w->y, need * 4)) || (rc = malloc_d(&w->dy, need * 4)) ||
        (rc = malloc_d(&w->Yb, need * 4)) ||
        (rc = malloc_d(&w->X, need * IN * 4)) ||
        (rc = malloc_d(&w->part, (size_t)((need + kColRows - 1) / kColRows) * HID * 8)) ||
        (rc = malloc_d(&w->lpart, (size_t)((need + 255) / 256) * 8))) {
        net_free_scratch(w);
        return rc;
    }
    w->cap = need;
    return CBLP_OK;
}

// forward over rpad rows of w->X (rows real): y, and the activations backward needs
int forward(wsnet* w, int64_t rows, int64_t rpad, hipStream_t s)
{
    hipLaunchKernelGGL(k_l1_fwd, dim3((unsigned)rpad), dim3(HID), 0, s, w->X, rows, w->P, w->z1,
                       w->h1b);
    // Z2 = H1 W2: B(k, n) = W2[k][n] = W2t[n][k], contiguous in k
    hipLaunchKernelGGL(k_gemm_rows<1>, dim3((unsigned)(rpad / 16)), dim3(256), 0, s, w->h1b,
                       w->W2t, w->z2, HID, HID, HID, HID, w->P + OFF_B2, w->h2);
    hipLaunchKernelGGL(k_l3_fwd, dim3((unsigned)((rpad + 3) / 4)), dim3(256), 0, s, w->h2, w->P,
                       rpad, w->y);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

int colsum(wsnet* w, const float* M, int64_t ld, int64_t rpad, int ncols, const float* sc,
           int64_t sst, float* out, hipStream_t s)
{
    const int nb = (int)((rpad + kColRows - 1) / kColRows);
    hipLaunchKernelGGL(k_colsum, dim3(nb), dim3(HID), 0, s, M, ld, rpad, ncols, sc, sst, w->part);
    hipLaunchKernelGGL(k_colsum_final, dim3((ncols + 255) / 256), dim3(256), 0, s, w->part, nb,
                       ncols, out);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

// loss and gradients into w->G for rows of (X, Y); X already in w->X
int backward(wsnet* w, const float* Y, int64_t rows, int64_t rpad, double* loss, hipStream_t s,
             double* loss_acc = nullptr)
{
    int rc;
    if ((rc = forward(w, rows, rpad, s))) return rc;
    const int lb = (int)((rpad + 255) / 256);
    hipLaunchKernelGGL(k_dy, dim3(lb), dim3(256), 0, s, w->y, Y, rows, rpad, w->dy, w->lpart);
    hipLaunchKernelGGL(k_l3_bwd, dim3((unsigned)rpad), dim3(HID), 0, s, w->dy, w->z2, w->P, w->dz2,
                       w->dz2b);
    // dW2 = H1^T dZ2 (K = rows), dH1 = dZ2 W2^T
    hipLaunchKernelGGL((k_gemm<true, false, 0>), dim3(HID / 64, HID / 16), dim3(256), 0, s, w->h1b,
                       w->dz2b, w->G + OFF_W2, HID, (int)rpad, HID, HID, nullptr, nullptr);
    // dH1 = dZ2 W2^T: B(k, n) = W2[n][k], contiguous in k
    hipLaunchKernelGGL(k_gemm_rows<0>, dim3((unsigned)(rpad / 16)), dim3(256), 0, s, w->dz2b,
                       w->W2b, w->dh1, HID, HID, HID, HID, nullptr, nullptr);
    hipLaunchKernelGGL(k_l1_bwd, dim3((unsigned)rpad), dim3(HID), 0, s, w->dh1, w->z1, w->dz1);
    MHIP(hipGetLastError());
    if ((rc = colsum(w, w->h2, HID, rpad, HID, w->dy, 1, w->G + OFF_W3, s))) return rc;
    if ((rc = colsum(w, w->dy, 1, rpad, 1, nullptr, 0, w->G + OFF_B3, s))) return rc;
    if ((rc = colsum(w, w->dz2, HID, rpad, HID, nullptr, 0, w->G + OFF_B2, s))) return rc;
    if ((rc = colsum(w, w->dz1, HID, rpad, HID, nullptr, 0, w->G + OFF_B1, s))) return rc;
    if (loss_acc) hipLaunchKernelGGL(k_loss_add, dim3(1), dim3(64), 0, s, w->lpart, lb, loss_acc);
    for (int k = 0; k < IN; ++k)
        if ((rc = colsum(w, w->dz1, HID, rpad, HID, w->X + k, IN, w->G + OFF_W1 + k * HID, s)))
            return rc;
    if (loss) {
        std::vector<double> lp(lb);
        MHIP(hipMemcpyAsync(lp.data(), w->lpart, lb * sizeof(double), hipMemcpyDeviceToHost, s));
        MHIP(hipStreamSynchronize(s));
        double acc = 0.0;
        for (double x : lp) acc += x;
        *loss = rows > 0 ? acc / (double)rows : 0.0;
    }
    return CBLP_OK;
}

int adam(wsnet* w, float lr, hipStream_t s)
{
    w->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)w->step), c2 = 1.0f - std::pow(b2, (float)w->step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((NPARAM + 255) / 256)), dim3(256), 0, s, w->P, w->G,
                       w->M, w->V, NPARAM, lr, b1, b2, 1e-8f, c1, c2);
    hipLaunchKernelGGL(k_round_w2, dim3(HID), dim3(HID), 0, s, w->P + OFF_W2, w->W2b, w->W2t);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

int load_rows(wsnet* w, const float* X, int64_t rows, int64_t rpad, hipStream_t s)
{
    MHIP(hipMemcpyAsync(w->X, X, (size_t)rows * IN * 4, hipMemcpyDeviceToDevice, s));
    if (rpad > rows) MHIP(hipMemsetAsync(w->X + rows * IN, 0, (size_t)(rpad - rows) * IN * 4, s));
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
    e = hipMemsetAsync(tail, 0, (size_t)3 * h->n * 8, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_feat_seg<T>, dim3(grid), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_feat_fold<T>, dim3((unsigned)((h->n + 255) / 256)), dim3(256), 0, s, a,
                           grid, (const T*)h->r, (const T*)h->c, mx, X);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(mx);
    (void)hipFree(part);
    (void)hipFree(tail);
    if (e != hipSuccess) return mfail(CBLP_EHIP, std::string("features: ") + hipGetErrorString(e));
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
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((rows + kInferRows - 1) / kInferRows)),
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
    if ((rc = ensure_scratch(w, rows))) return rc;
    const int64_t rpad = pad16(rows);
    if ((rc = load_rows(w, X, rows, rpad, s))) return rc;
    if ((rc = backward(w, Y, rows, rpad, loss, s))) return rc;
    if (grads) MHIP(hipMemcpyAsync(grads, w->G, NPARAM * 4, hipMemcpyDeviceToDevice, s));
    MHIP(hipStreamSynchronize(s));
    return CBLP_OK;
}

int wsnet_train_step(wsnet_t w, const float* X, const float* Y, int64_t rows, float lr,
                     double* loss, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !X || !Y || rows < 1 || !(lr > 0.0f)) return mfail(CBLP_EINVAL, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ensure_scratch(w, rows))) return rc;
    const int64_t rpad = pad16(rows);
    if ((rc = load_rows(w, X, rows, rpad, s))) return rc;
    if ((rc = backward(w, Y, rows, rpad, loss, s))) return rc;
    return adam(w, lr, s);
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
    if ((rc = ensure_scratch(w, batch))) return rc;
    int32_t* perm = nullptr;
    double* acc = nullptr;
    if ((rc = malloc_d(&perm, (size_t)rows * 4)) || (rc = malloc_d(&acc, 8))) {
        if (perm) (void)hipFree(perm);
        return rc;
    }
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
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, acc, (int64_t)1, 0.0);
        for (int64_t b0 = 0; b0 < rows && rc == CBLP_OK; b0 += batch) {
            const int64_t cnt = std::min(batch, rows - b0);
            const int64_t rpad = pad16(cnt);
            hipLaunchKernelGGL(k_gather, dim3((unsigned)((rpad + 255) / 256)), dim3(256), 0, s, X, Y,
                               perm + b0, cnt, rpad, w->X, w->Yb);
            // each batch's mean loss weighted by its rows: acc gets sum of squared errors
            if ((rc = backward(w, w->Yb, cnt, rpad, nullptr, s, acc))) break;
            rc = adam(w, lr, s);
        }
        if (rc) break;
        double h = 0.0;
        if (hipMemcpyAsync(&h, acc, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = mfail(CBLP_EHIP, "reading the epoch loss failed");
            break;
        }
        if (losses) losses[e] = h / (double)rows;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(perm);
    (void)hipFree(acc);
    return rc;
}

int wsnet_targets(cblp_t h, const void* eta, float* Y, void* stream)
{
    set_error(CBLP_OK, "");
    if (!h || !eta || !Y) return mfail(CBLP_EINVAL, "NULL argument");
    if (h->a_ptr) return mfail(CBLP_EINVAL, "warm start needs the identity resource matrix");
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = (unsigned)((h->n + 255) / 256);
    if (h->dtype == CBLP_F32)
        hipLaunchKernelGGL(k_targets<float>, dim3(g), dim3(256), 0, s, (const float*)eta,
                           (const float*)h->r, h->n, Y);
    else
        hipLaunchKernelGGL(k_targets<double>, dim3(g), dim3(256), 0, s, (const double*)eta,
                           (const double*)h->r, h->n, Y);
    MHIP(hipGetLastError());
    return CBLP_OK;
}

int wsnet_predict(wsnet_t w, cblp_t h, void* eta, void* stream)
{
    set_error(CBLP_OK, "");
    if (!w || !h || !eta) return mfail(CBLP_EINVAL, "NULL argument");
    if (h->a_ptr) return mfail(CBLP_EINVAL, "warm start needs the identity resource matrix");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = ensure_scratch(w, h->n))) return rc;
    rc = h->dtype == CBLP_F32 ? features_impl<float>(h, w->X, s) : features_impl<double>(h, w->X, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((h->n + kInferRows - 1) / kInferRows)),
                       dim3(256), 0, s, w->X, h->n,
                       w->P, w->W2t, w->y);
    const unsigned g = (unsigned)((h->n + 255) / 256);
    if (h->dtype == CBLP_F32)
        hipLaunchKernelGGL(k_eta_from_y<float>, dim3(g), dim3(256), 0, s, w->y, (const float*)h->r,
                           h->n, (float*)eta);
    else
        hipLaunchKernelGGL(k_eta_from_y<double>, dim3(g), dim3(256), 0, s, w->y, (const double*)h->r,
                           h->n, (double*)eta);
    MHIP(hipGetLastError());
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

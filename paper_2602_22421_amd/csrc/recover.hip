// SBLP -> CBLP recovery (Section 4.4, the recovery lemma, in its GAM form):
// from per-entry sales y (the caller's CSR order) the nested assortments of
// each segment and the probability of offering each.
//
// A segment's products are ordered by key = y_lj / v_lj, decreasing, ties by
// CSR position; S_q is the set of the first q of them.  Offering S_q for a
// share x_q of the time sells x_q v_j / (vt0 + sum_{S_q} vt) of each j in
// S_q, so x_q = (key_q - key_{q+1}) (vt0 + sum_{S_q} vt) reproduces y; the
// probability is x_q / lambda and the empty set takes the rest.
//
// k_recover: one wave per segment.  The row is staged in LDS 64 entries at
// a time (key = y / v and v - w); each lane takes entries of the row and
// finds, by one pass over the staged chunks, its entry's rank, the
// attraction sum of the entries ranked at or before it and the next key.
// The chunk reads are LDS broadcasts, so the pass costs k LDS reads per lane
// and no global load after the staging.
#include <string>

#include "common.hpp"
#include "handle.hpp"

namespace cblp {
namespace {

constexpr int kRecWaves = 4;

template <typename T>
__global__ void __launch_bounds__(64 * kRecWaves) k_recover(int64_t L, const int64_t* seg_ptr,
                                                            const T* v, const T* w, const T* v0,
                                                            const T* lam, const double* y,
                                                            int32_t* rank, double* alpha,
                                                            double* alpha0)
{
    __shared__ double skey[kRecWaves][64], sdv[kRecWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t l = (int64_t)blockIdx.x * kRecWaves + wv;
    if (l >= L) return;   // the whole wave: no block-wide barrier follows
    double* sk = skey[wv];
    double* sd = sdv[wv];
    const int64_t b = seg_ptr[l], k = seg_ptr[l + 1] - b;
    // the row's entries are staged in LDS 64 at a time; the wave barriers
    // keep a chunk's reads before the next chunk's writes
    double vt0 = (double)v0[l];
    for (int64_t p0 = 0; p0 < k; p0 += 64) {
        __builtin_amdgcn_wave_barrier();
        if (p0 + lane < k) sd[lane] = (double)w[b + p0 + lane];
        __builtin_amdgcn_wave_barrier();
        const int kc = (int)(k - p0 < 64 ? k - p0 : 64);
        for (int t = 0; t < kc; ++t) vt0 += sd[t];   // in row order, the same on every lane
    }
    const double la = (double)lam[l];
    double tot = 0.0;
    for (int64_t q0 = 0; q0 < k; q0 += 64) {
        const int64_t q = q0 + lane;
        const bool mine = q < k;
        const double key = mine ? y[b + q] / (double)v[b + q] : 0.0;
        int32_t r = 0;
        double W = vt0, next = 0.0;
        for (int64_t p0 = 0; p0 < k; p0 += 64) {
            __builtin_amdgcn_wave_barrier();
            const int64_t pl = p0 + lane;
            if (pl < k) {
                sk[lane] = y[b + pl] / (double)v[b + pl];
                sd[lane] = (double)v[b + pl] - (double)w[b + pl];
            }
            __builtin_amdgcn_wave_barrier();
            const int kc = (int)(k - p0 < 64 ? k - p0 : 64);
            for (int t = 0; t < kc; ++t) {
                const int64_t p = p0 + t;
                const double kp = sk[t];
                const bool before = kp > key || (kp == key && p < q);
                if (before) ++r;
                if (before || p == q) W += sd[t];
                else next = fmax(next, kp);   // ranked after q: the largest is the next key
            }
        }
        if (mine) {
            const double a = la > 0.0 ? (key - next) * W / la : 0.0;
            rank[b + q] = r;
            alpha[b + q] = a;
            tot += a;
        }
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_down(tot, o, 64);
    if (lane == 0) alpha0[l] = la > 0.0 ? 1.0 - tot : 1.0;
}

}  // namespace
}  // namespace cblp

using namespace cblp;

extern "C" int cblp_recover(cblp_t h, const double* y, int32_t* rank, double* alpha,
                            double* alpha0, void* stream)
{
    set_error(CBLP_OK, "");
    if (!h || !y || !rank || !alpha || !alpha0) return set_error(CBLP_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    if (h->L > 0) {
        const unsigned grid = (unsigned)((h->L + kRecWaves - 1) / kRecWaves);
        if (h->dtype == CBLP_F32)
            hipLaunchKernelGGL(k_recover<float>, dim3(grid), dim3(64 * kRecWaves), 0, s, h->L, h->seg_ptr,
                               (const float*)h->v, (const float*)h->w, (const float*)h->v0,
                               (const float*)h->lam, y, rank, alpha, alpha0);
        else
            hipLaunchKernelGGL(k_recover<double>, dim3(grid), dim3(64 * kRecWaves), 0, s, h->L, h->seg_ptr,
                               (const double*)h->v, (const double*)h->w, (const double*)h->v0,
                               (const double*)h->lam, y, rank, alpha, alpha0);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CBLP_EHIP, std::string("recover: ") + hipGetErrorString(e));
    return CBLP_OK;
}

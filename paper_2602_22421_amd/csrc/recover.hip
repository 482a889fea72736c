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
// k_recover: one wave per segment; each lane takes entries of the row and
// finds, by one pass over the row, the entry's rank, the attraction sum of
// the entries ranked at or before it and the next key.
#include <string>

#include "common.hpp"
#include "handle.hpp"

namespace cblp {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) k_recover(int64_t L, const int64_t* seg_ptr, const T* v,
                                                 const T* w, const T* v0, const T* lam,
                                                 const double* y, int32_t* rank, double* alpha,
                                                 double* alpha0)
{
    const int lane = threadIdx.x & 63;
    const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (l >= L) return;
    const int64_t b = seg_ptr[l], k = seg_ptr[l + 1] - b;
    double vt0 = (double)v0[l];
    for (int64_t q = 0; q < k; ++q) vt0 += (double)w[b + q];
    const double la = (double)lam[l];
    double tot = 0.0;
    for (int64_t q = lane; q < k; q += 64) {
        const double key = y[b + q] / (double)v[b + q];
        int32_t r = 0;
        double W = vt0, next = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            const double kp = y[b + p] / (double)v[b + p];
            const bool before = kp > key || (kp == key && p < q);
            if (before) ++r;
            if (before || p == q) W += (double)v[b + p] - (double)w[b + p];
            else next = fmax(next, kp);   // ranked after q: the largest is the next key
        }
        const double a = la > 0.0 ? (key - next) * W / la : 0.0;
        rank[b + q] = r;
        alpha[b + q] = a;
        tot += a;
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
        const unsigned grid = (unsigned)((h->L + 3) / 4);
        if (h->dtype == CBLP_F32)
            hipLaunchKernelGGL(k_recover<float>, dim3(grid), dim3(256), 0, s, h->L, h->seg_ptr,
                               (const float*)h->v, (const float*)h->w, (const float*)h->v0,
                               (const float*)h->lam, y, rank, alpha, alpha0);
        else
            hipLaunchKernelGGL(k_recover<double>, dim3(grid), dim3(256), 0, s, h->L, h->seg_ptr,
                               (const double*)h->v, (const double*)h->w, (const double*)h->v0,
                               (const double*)h->lam, y, rank, alpha, alpha0);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CBLP_EHIP, std::string("recover: ") + hipGetErrorString(e));
    return CBLP_OK;
}

// Time reconstruction of the modes (section 2.4, step 4, Eq. sol_reconstruct).
//
// For real boundary data the coefficients of negative frequencies are the
// conjugates of the positive ones (Eq. SCVS_bc), so the real field is
//   u(t) = sum_k c_k Re(u_k exp(j w_k t)),  c_k = 1 for w_k = 0, else 2.
// Each workgroup owns 256 values x TT times; the twiddles exp(j w_k t_n) of
// its time tile are computed once into LDS, so every mode value is read once
// per time tile and every output is written once (an HBM-streaming kernel).
#include "internal.hpp"

namespace scvs {
namespace {

constexpr int TT = 16;  // times per workgroup
constexpr int KT = 64;  // modes per LDS twiddle tile

__global__ void __launch_bounds__(256) k_synth(int64_t nk, const double* __restrict__ omega,
                                               const double2* __restrict__ modes, int64_t nvals, int64_t nt,
                                               const double* __restrict__ times, double* __restrict__ out) {
  __shared__ double2 tw[KT][TT];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t0 = (int64_t)blockIdx.y * TT;
  double acc[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) acc[t] = 0.0;
  for (int64_t k0 = 0; k0 < nk; k0 += KT) {
    __syncthreads();
    for (int p = threadIdx.x; p < KT * TT; p += blockDim.x) {
      const int kk = p / TT, tt = p % TT;
      const int64_t k = k0 + kk, tn = t0 + tt;
      double sv = 0.0, cv = 0.0;
      if (k < nk && tn < nt) {
        const double w = omega[k];
        sincos(w * times[tn], &sv, &cv);
        const double f = (w == 0.0) ? 1.0 : 2.0;
        sv *= f;
        cv *= f;
      }
      tw[kk][tt] = make_double2(cv, sv);
    }
    __syncthreads();
    if (i < nvals) {
      const int64_t kmax = (nk - k0) < KT ? (nk - k0) : KT;
      for (int64_t kk = 0; kk < kmax; ++kk) {
        const double2 u = modes[(k0 + kk) * nvals + i];
#pragma unroll
        for (int t = 0; t < TT; ++t) acc[t] += u.x * tw[kk][t].x - u.y * tw[kk][t].y;
      }
    }
  }
  if (i < nvals) {
#pragma unroll
    for (int t = 0; t < TT; ++t)
      if (t0 + t < nt) out[(t0 + t) * nvals + i] = acc[t];
  }
}

}  // namespace

void synthesize(hipStream_t s, int64_t nk, const double* omega, const double2* modes, int64_t nvals, int64_t nt,
                const double* times, double* out) {
  if (nvals == 0 || nt == 0) return;
  DBuf<double> om, tm;
  om.upload(omega, nk, s);
  tm.upload(times, nt, s);
  dim3 g((unsigned)((nvals + 255) / 256), (unsigned)((nt + TT - 1) / TT));
  k_synth<<<g, 256, 0, s>>>(nk, om, modes, nvals, nt, tm, out);
  SCVS_HIP(hipGetLastError());
  SCVS_HIP(hipStreamSynchronize(s));
}

}  // namespace scvs

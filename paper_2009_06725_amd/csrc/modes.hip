// Mode selection (section 2.4, step 2 and the closing remarks): the a-priori
// truncation error of the boundary data, Eq. mode_error, and the a-posteriori
// change of the reconstructed solution when one more mode is added.
//
// For real periodic data with two-sided coefficients (zeroth mode once, every
// other mode twice), Parseval turns the L2(Gamma x T) norms of Eq. mode_error
// into sums over the modes of T * w_k * ||data_k||^2_{L2(Gamma)} with w_0 = 1 and
// w_k = 2, and the change from adding mode N to the reconstruction, Eq.
// sol_reconstruct, into T * w_N * ||u_N||^2_{L2(Omega)}. The device computes the
// per-mode norms; the selection itself is host arithmetic.
#include <mutex>
#include <numeric>

#include "internal.hpp"

namespace scvs {
namespace {

// Per boundary facet: its area, and for every system the integral of |g_h|^2
// over it (g_h the quadratic interpolant of the nodal data in xs); out_area[f],
// out_g[s][f]. Degree-5 facet quadrature on the quadratic facet map.
template <int D>
__global__ void k_facet_l2(const int32_t* __restrict__ fnodes, int64_t nf, const double* __restrict__ xyz,
                           const double* __restrict__ exyz, int64_t nv, const double* __restrict__ qb,
                           const double* __restrict__ qw, int nq, const double2* __restrict__ xs, int64_t xst,
                           int nsys, double* __restrict__ out_area, double* __restrict__ out_g) {
  constexpr int NFV = D, NFN = D * (D + 1) / 2;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double X[NFN][D];
  int32_t nd[NFN];
#pragma unroll
  for (int a = 0; a < NFN; ++a) {
    nd[a] = fnodes[f * NFN + a];
#pragma unroll
    for (int k = 0; k < D; ++k)
      X[a][k] = (nd[a] < nv) ? xyz[(int64_t)nd[a] * D + k] : exyz[(int64_t)(nd[a] - nv) * D + k];
  }
  const int le[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  double area = 0.0;
  for (int s = -1; s < nsys; ++s) {  // s = -1: the area pass
    double acc = 0.0;
    for (int q = 0; q < nq; ++q) {
      double mu[NFV];
#pragma unroll
      for (int k = 0; k < NFV; ++k) mu[k] = qb[q * NFV + k];
      double psi[NFN], dmu[NFN][NFV];
#pragma unroll
      for (int a = 0; a < NFN; ++a)
#pragma unroll
        for (int k = 0; k < NFV; ++k) dmu[a][k] = 0.0;
#pragma unroll
      for (int k = 0; k < NFV; ++k) {
        psi[k] = mu[k] * (2.0 * mu[k] - 1.0);
        dmu[k][k] = 4.0 * mu[k] - 1.0;
      }
#pragma unroll
      for (int e = 0; e < NFN - NFV; ++e) {
        const int i = le[e][0], j = le[e][1];
        psi[NFV + e] = 4.0 * mu[i] * mu[j];
        dmu[NFV + e][i] = 4.0 * mu[j];
        dmu[NFV + e][j] = 4.0 * mu[i];
      }
      double T[D - 1][D];
#pragma unroll
      for (int t = 0; t < D - 1; ++t)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double sum = 0.0;
#pragma unroll
          for (int a = 0; a < NFN; ++a) sum += X[a][k] * (dmu[a][t + 1] - dmu[a][0]);
          T[t][k] = sum;
        }
      double J;
      if constexpr (D == 2) {
        J = sqrt(T[0][0] * T[0][0] + T[0][1] * T[0][1]);
      } else {
        const double n0 = T[0][1] * T[1][2] - T[0][2] * T[1][1];
        const double n1 = T[0][2] * T[1][0] - T[0][0] * T[1][2];
        const double n2 = T[0][0] * T[1][1] - T[0][1] * T[1][0];
        J = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
      }
      if (s < 0) {
        acc += qw[q] * J;
      } else {
        const double2* x = xs + (int64_t)s * xst;
        double v2 = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          double2 gv = make_double2(0.0, 0.0);
#pragma unroll
          for (int a = 0; a < NFN; ++a) {
            const double2 xa = x[(int64_t)nd[a] * D + c];
            gv.x += psi[a] * xa.x;
            gv.y += psi[a] * xa.y;
          }
          v2 += gv.x * gv.x + gv.y * gv.y;
        }
        acc += qw[q] * J * v2;
      }
    }
    if (s < 0)
      area = acc;
    else
      out_g[(int64_t)s * nf + f] = acc;
  }
  out_area[f] = area;
}

// Block partial sums of u^H (I_d (x) M) u and p^H Mp p for every system. A wavefront
// walks one row of the quadratic pattern at a time, loading each (col, M) slot once for
// all systems: its lanes are (system, component) pairs p = s*D + c (UL = 64/D*D pairs per
// pass, further passes when the batch has more). Pair lane p accumulates
// Re(conj(u_s[A][c]) (M u_s^c)_A) over its rows; each block then sums its waves and the
// components of a system in a fixed order into part_u[s][block]. The pressure part is a
// plain per-vertex sum per system. Block partials are reduced in block order by
// k_sum_parts, so the norms are bit-reproducible.
constexpr int NB_L2 = 256;  // blocks (partials per system)
template <int D>
__global__ void __launch_bounds__(256) k_mode_l2(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                 const double* __restrict__ M, const double* __restrict__ Mp,
                                                 int64_t n2, int64_t nv, const double2* __restrict__ u, int64_t ust,
                                                 const double2* __restrict__ p, int64_t pst, int nsys,
                                                 double* __restrict__ part_u, double* __restrict__ part_p) {
  __shared__ double sh[256];
  constexpr int UL = (64 / D) * D;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * 4, w0 = (int64_t)blockIdx.x * 4 + wave;
  const int npair = nsys * D;
  for (int base = 0; base < npair; base += UL) {
    const int pr = base + lane;
    const bool ok = lane < UL && pr < npair;
    const int si = ok ? pr / D : 0, c = ok ? pr % D : 0;
    const double2* __restrict__ us = u + (int64_t)si * ust;
    double acc = 0.0;
    for (int64_t A = w0; A < n2; A += nw) {
      const int64_t j0 = rowptr[A], j1 = rowptr[A + 1];
      double2 mu = make_double2(0.0, 0.0);
      for (int64_t jb = j0; jb < j1; jb += 64) {
        const int n = (int)min((int64_t)64, j1 - jb);
        int32_t mc = 0;
        double mv = 0.0;
        if (lane < n) {
          mc = col[jb + lane];
          mv = M[jb + lane];
        }
        for (int t = 0; t < n; ++t) {
          const int32_t B = __shfl(mc, t, 64);
          const double w = __shfl(mv, t, 64);
          if (ok) {
            const double2 v = us[(int64_t)B * D + c];
            mu.x += w * v.x;
            mu.y += w * v.y;
          }
        }
      }
      if (ok) {
        const double2 ua = us[A * D + c];
        acc += ua.x * mu.x + ua.y * mu.y;
      }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    const int nsp = min(UL, npair - base) / D;  // systems in this pass
    if (threadIdx.x < nsp) {
      double t = 0.0;
      for (int w = 0; w < 4; ++w)
        for (int cc = 0; cc < D; ++cc) t += sh[w * 64 + threadIdx.x * D + cc];
      part_u[(int64_t)(base / D + threadIdx.x) * gridDim.x + blockIdx.x] = t;
    }
    __syncthreads();
  }
  for (int si = 0; si < nsys; ++si) {
    const double2* __restrict__ ps = p + (int64_t)si * pst;
    double ap = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += (int64_t)gridDim.x * blockDim.x) {
      const double2 pa = ps[v];
      ap += Mp[v] * (pa.x * pa.x + pa.y * pa.y);
    }
    sh[threadIdx.x] = ap;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part_p[(int64_t)si * gridDim.x + blockIdx.x] = sh[0];
    __syncthreads();
  }
}

// out[s] = sum of part[s][0..nb) in block order, for s < n.
__global__ void k_sum_parts(const double* __restrict__ part, int nb, int n, double* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[(int64_t)s * nb + b];
  out[s] = t;
}

// The norms of nsys systems with all partials and sums in `work` (2*nsys*NB_L2 + 2*nsys
// doubles on the device); un2/pn2 are host outputs.
void mode_norms_into(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* work, double* un2,
                     double* pn2) {
  hipStream_t s = m->ctx->stream;
  const int D = m->dim;
  double* pu = work;
  double* pp = work + nsys * NB_L2;
  double* su = work + 2 * nsys * NB_L2;
  double* sp = su + nsys;
  const unsigned nb = NB_L2;
  if (D == 2)
    k_mode_l2<2><<<nb, 256, 0, s>>>(m->rowptr, m->col, m->M, m->Mp, m->n2, m->nv, (const double2*)u, m->n2 * D,
                                    (const double2*)p, m->nv, (int)nsys, pu, pp);
  else
    k_mode_l2<3><<<nb, 256, 0, s>>>(m->rowptr, m->col, m->M, m->Mp, m->n2, m->nv, (const double2*)u, m->n2 * D,
                                    (const double2*)p, m->nv, (int)nsys, pu, pp);
  const unsigned ns = (unsigned)((nsys + 63) / 64);
  k_sum_parts<<<ns, 64, 0, s>>>(pu, NB_L2, (int)nsys, su);
  k_sum_parts<<<ns, 64, 0, s>>>(pp, NB_L2, (int)nsys, sp);
  launch_check(s);
  SCVS_HIP(hipMemcpyAsync(un2, su, sizeof(double) * nsys, hipMemcpyDeviceToHost, s));
  SCVS_HIP(hipMemcpyAsync(pn2, sp, sizeof(double) * nsys, hipMemcpyDeviceToHost, s));
  SCVS_HIP(hipStreamSynchronize(s));
}

}  // namespace

void boundary_norms(scvs_mesh m, int64_t nsys, const double* traction, const void* g, double* hn2, double* gn2) {
  hipStream_t s = m->ctx->stream;
  const int D = m->dim;
  const int64_t ndof = D * m->n2 + m->nv;
  const int ntr = (int)m->traction_tags.size();
  for (int64_t k = 0; k < nsys; ++k) hn2[k] = gn2[k] = 0.0;
  if (m->nf == 0) return;
  // nodal boundary data of every system: g on Dirichlet nodes, zero elsewhere (walls too)
  DBuf<double2> xg;
  DBuf<int> act;
  std::vector<int> a(nsys);
  std::iota(a.begin(), a.end(), 0);
  act.upload(a.data(), nsys, s);
  xg.alloc((size_t)nsys * ndof);
  scatter_dirichlet(m, nsys, g, VArg{xg.p, ndof}, act, s);
  std::vector<double> qb, qw;
  gm_rule(D - 1, 2, qb, qw);
  DBuf<double> dqb, dqw, area, gf;
  dqb.upload(qb.data(), qb.size(), s);
  dqw.upload(qw.data(), qw.size(), s);
  area.alloc(m->nf);
  gf.alloc((size_t)nsys * m->nf);
  const unsigned nb = (unsigned)((m->nf + 255) / 256);
  if (D == 2)
    k_facet_l2<2><<<nb, 256, 0, s>>>(m->fnodes, m->nf, m->xyz, m->exyz, m->nv, dqb, dqw, (int)qw.size(), xg, ndof,
                                     (int)nsys, area, gf);
  else
    k_facet_l2<3><<<nb, 256, 0, s>>>(m->fnodes, m->nf, m->xyz, m->exyz, m->nv, dqb, dqw, (int)qw.size(), xg, ndof,
                                     (int)nsys, area, gf);
  launch_check(s);
  std::vector<double> ha(m->nf), hg((size_t)nsys * m->nf);
  std::vector<int32_t> tags(m->nf);
  download(ha.data(), area.p, m->nf, s);
  download(hg.data(), gf.p, (size_t)nsys * m->nf, s);
  download(tags.data(), m->btags.p, m->nf, s);
  // facet kinds by tag; sums in facet order (deterministic)
  auto kind_of = [&](int32_t tag) {
    for (size_t k = 0; k < m->bc_tags.size(); ++k)
      if (m->bc_tags[k] == tag) return m->bc_kinds[k];
    return (int32_t)SCVS_BC_FREE;
  };
  std::vector<double> tarea(ntr, 0.0);
  for (int64_t f = 0; f < m->nf; ++f) {
    const int32_t kd = kind_of(tags[f]);
    if (kd == SCVS_BC_DIRICHLET)
      for (int64_t k = 0; k < nsys; ++k) gn2[k] += hg[(size_t)k * m->nf + f];
    if (kd == SCVS_BC_TRACTION)
      for (int t = 0; t < ntr; ++t)
        if (m->traction_tags[t] == tags[f]) tarea[t] += ha[f];
  }
  // h = -P n per traction tag: int |h|^2 = |P|^2 * area
  for (int64_t k = 0; k < nsys; ++k)
    for (int t = 0; t < ntr; ++t) {
      const double pr = traction[2 * (k * ntr + t)], pi = traction[2 * (k * ntr + t) + 1];
      hn2[k] += (pr * pr + pi * pi) * tarea[t];
    }
}

void mode_norms(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2) {
  DBuf<double> work;
  work.alloc((size_t)nsys * (2 * NB_L2 + 2));
  mode_norms_into(m, nsys, u, p, work.p, un2, pn2);
}

// ---- mode norms without allocation ----
// The partial sums of up to SCVS_NOALLOC_MAX_SYSTEMS systems live in this file-scope
// device array (one copy per GPU, held until the process ends). Host code never passes
// the array's name to a kernel: it uses the device address that hipGetSymbolAddress
// returned for the current GPU when a context was created there.
static __device__ __align__(256) double scratch[(size_t)SCVS_NOALLOC_MAX_SYSTEMS * (2 * NB_L2 + 2)];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

void noalloc_init(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return;  // the entry point then reports it
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  SCVS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  SCVS_REQUIRE(ptr != nullptr, SCVS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr[device] = ptr;
}

void mode_norms_noalloc(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2) {
  SCVS_REQUIRE(nsys <= SCVS_NOALLOC_MAX_SYSTEMS, SCVS_E_CAPACITY,
               "at most " + std::to_string(SCVS_NOALLOC_MAX_SYSTEMS) + " systems per call without allocation");
  const int dev = m->ctx->device;
  void* ptr = nullptr;
  if (dev >= 0 && dev < SCRATCH_MAX_DEVICES) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ptr = g_scratch_ptr[dev];
  }
  SCVS_REQUIRE(ptr != nullptr, SCVS_E_STATE, "no scratch array address for this device");
  mode_norms_into(m, nsys, u, p, static_cast<double*>(ptr), un2, pn2);
}

}  // namespace scvs

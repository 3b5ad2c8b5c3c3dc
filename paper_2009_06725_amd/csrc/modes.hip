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

// Block partial sums of u^H (I_d (x) M) u and p^H Mp p for system blockIdx.y.
template <int D>
__global__ void __launch_bounds__(256) k_mode_l2(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                                                 const double* __restrict__ M, const double* __restrict__ Mp,
                                                 int64_t n2, int64_t nv, const double2* __restrict__ u, int64_t ust,
                                                 const double2* __restrict__ p, int64_t pst,
                                                 double* __restrict__ part_u, double* __restrict__ part_p) {
  __shared__ double shu[256], shp[256];
  const int s = blockIdx.y;
  const double2* us = u + (int64_t)s * ust;
  const double2* ps = p + (int64_t)s * pst;
  double au = 0.0, ap = 0.0;
  for (int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; A < n2; A += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      double2 mu = make_double2(0.0, 0.0);
      for (int64_t j = rowptr[A]; j < rowptr[A + 1]; ++j) {
        const double2 v = us[(int64_t)col[j] * D + c];
        mu.x += M[j] * v.x;
        mu.y += M[j] * v.y;
      }
      const double2 ua = us[A * D + c];
      au += ua.x * mu.x + ua.y * mu.y;  // Re(conj(u_A) (M u)_A)
    }
    if (A < nv) {
      const double2 pa = ps[A];
      ap += Mp[A] * (pa.x * pa.x + pa.y * pa.y);
    }
  }
  shu[threadIdx.x] = au;
  shp[threadIdx.x] = ap;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      shu[threadIdx.x] += shu[threadIdx.x + o];
      shp[threadIdx.x] += shp[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_u[(int64_t)s * gridDim.x + blockIdx.x] = shu[0];
    part_p[(int64_t)s * gridDim.x + blockIdx.x] = shp[0];
  }
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
  hipStream_t s = m->ctx->stream;
  const int D = m->dim;
  const unsigned nb = 256;
  DBuf<double> pu, pp;
  pu.alloc((size_t)nsys * nb);
  pp.alloc((size_t)nsys * nb);
  const dim3 gr(nb, (unsigned)nsys);
  if (D == 2)
    k_mode_l2<2><<<gr, 256, 0, s>>>(m->rowptr, m->col, m->M, m->Mp, m->n2, m->nv, (const double2*)u, m->n2 * D,
                                    (const double2*)p, m->nv, pu, pp);
  else
    k_mode_l2<3><<<gr, 256, 0, s>>>(m->rowptr, m->col, m->M, m->Mp, m->n2, m->nv, (const double2*)u, m->n2 * D,
                                    (const double2*)p, m->nv, pu, pp);
  launch_check(s);
  std::vector<double> hu((size_t)nsys * nb), hp((size_t)nsys * nb);
  download(hu.data(), pu.p, hu.size(), s);
  download(hp.data(), pp.p, hp.size(), s);
  for (int64_t k = 0; k < nsys; ++k) {
    double a = 0.0, b = 0.0;
    for (unsigned i = 0; i < nb; ++i) {
      a += hu[(size_t)k * nb + i];
      b += hp[(size_t)k * nb + i];
    }
    un2[k] = a;
    pn2[k] = b;
  }
}

}  // namespace scvs

// Multi-system complex SpMV and the block preconditioner (section 2.3, Eq. linear_sys_def).
//
// One row of the quadratic-node pattern S2 serves every velocity component
// and every system of a batch: a wavefront walks the row once, loading each
// (col, Ks, M) slot a single time, and its lanes are (system, component)
// pairs that gather x[col][c] of their own system. For a vertex row the same
// gathered values feed the divergence row G^T (the transposed pattern of C21
// is the vertex row of S2); the vertex-column prefix of each row carries G.
//
// Per system the momentum block is mu Ks + j w rho M; the preconditioner uses
// the real shift mu Ks + |w| rho M and the pressure Laplacian G^T diag(M)^-1 G.
#include "internal.hpp"

namespace scvs {
namespace {

struct LaneMap {
  int G;     // (system, component) pairs per row
  int Geff;  // lanes used per row group (a multiple of D)
  int R;     // rows per wavefront
  int iters; // passes over the pairs
};

LaneMap lane_map(int nact, int D) {
  const int G = nact * D, UL = (64 / D) * D;
  if (G <= UL) return {G, G, UL / G, 1};
  return {G, UL, 1, (G + UL - 1) / UL};
}

struct MeshArgs {
  int64_t n2, nv, nnz21, nnzv;
  const int64_t *rowptr, *rowptr21;
  const int32_t *col, *nvc, *dmask;
  const double *Ks, *M, *G, *Gt, *Kd, *Md, *Mp, *lpdinv;
  double mu, rho, lpmax;
};

MeshArgs mesh_args(scvs_mesh m) {
  MeshArgs a;
  a.n2 = m->n2;
  a.nv = m->nv;
  a.nnz21 = m->nnz21;
  a.nnzv = m->nnzv;
  a.rowptr = m->rowptr;
  a.rowptr21 = m->rowptr21;
  a.col = m->col;
  a.nvc = m->nvc;
  a.dmask = m->dmask;
  a.Ks = m->Ks;
  a.M = m->M;
  a.G = m->G;
  a.Gt = m->Gt;
  a.Kd = m->Kd;
  a.Md = m->Md;
  a.Mp = m->Mp;
  a.lpdinv = m->lpdinv;
  a.mu = m->mu;
  a.rho = m->rho;
  a.lpmax = m->lp_lmax;
  return a;
}

struct Lane {
  int64_t row;
  int p0;
  bool rowok;
};

__device__ __forceinline__ Lane lane_of(const LaneMap& lm, int64_t nrows) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rs = lane / lm.Geff;
  Lane L;
  L.p0 = lane % lm.Geff;
  L.row = ((int64_t)blockIdx.x * 4 + wave) * lm.R + rs;
  L.rowok = (rs < lm.R) && (L.row < nrows);
  return L;
}

__device__ __forceinline__ double in_scale(const Batch& b, int slot) {
  return b.insc ? b.insc[(int64_t)slot * b.insc_st + b.insc_idx] : 1.0;
}

// Sum over the D lanes of one system (lanes p = s*D + c are adjacent).
template <int D>
__device__ __forceinline__ double2 sum_components(double2 v) {
  double2 r = v;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    r.x += __shfl_down(v.x, k, 64);
    r.y += __shfl_down(v.y, k, 64);
  }
  return r;
}

template <int D, int MODE, bool MASK>
__global__ void __launch_bounds__(256) k_full(MeshArgs ma, Batch b, LaneMap lm, VArg x, VArg y, VArg f,
                                              const double* __restrict__ loads, int ntr,
                                              const double2* __restrict__ trac) {
  const Lane L = lane_of(lm, ma.n2);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.p0 + it * lm.Geff;
    const bool ok = L.rowok && p < lm.G;
    const int si = p / D, c = p % D;
    double2 au = make_double2(0.0, 0.0), ap = make_double2(0.0, 0.0);
    int slot = 0;
    double sc = 1.0;
    int32_t dm = 0;
    const int64_t A = L.row;
    if (ok) {
      slot = b.act[si];
      sc = in_scale(b, slot);
      const double2* __restrict__ xs = x.at(slot);
      const double wr = b.omega[slot] * ma.rho;
      dm = ma.dmask[A];
      const bool isv = A < ma.nv;
      const int64_t j0 = ma.rowptr[A], j1 = ma.rowptr[A + 1];
      if (dm == 0 || isv) {
        for (int64_t j = j0; j < j1; ++j) {
          const int32_t B = ma.col[j];
          if (MASK && ma.dmask[B] != 0) continue;
          const double2 xv = xs[(int64_t)B * D + c];
          if (dm == 0) {
            const double kr = ma.mu * ma.Ks[j], mi = wr * ma.M[j];
            au.x += kr * xv.x - mi * xv.y;
            au.y += kr * xv.y + mi * xv.x;
          }
          if (isv) {
            const double g = ma.Gt[(int64_t)c * ma.nnzv + j];
            ap.x += g * xv.x;
            ap.y += g * xv.y;
          }
        }
      }
      if (dm == 0) {
        const int nvr = ma.nvc[A];
        const int64_t o21 = ma.rowptr21[A];
        const double2* __restrict__ xp = xs + D * ma.n2;
        for (int jj = 0; jj < nvr; ++jj) {
          const double g = ma.G[(int64_t)c * ma.nnz21 + o21 + jj];
          const double2 pv = xp[ma.col[j0 + jj]];
          au.x += g * pv.x;
          au.y += g * pv.y;
        }
      }
      double2 yu;
      if (dm != 0) {
        const double2 xv = xs[A * D + c];
        yu = cscale(xv, sc);
        if (MODE == SPMV_RESID) yu = csub(f.at(slot)[A * D + c], yu);
      } else {
        au = cscale(au, sc);
        if (MODE == SPMV_APPLY) {
          yu = au;
        } else if (MODE == SPMV_RESID) {
          yu = csub(f.at(slot)[A * D + c], au);
        } else {
          yu = make_double2(-au.x, -au.y);
          for (int t = 0; t < ntr; ++t) {
            const double2 P = trac[(int64_t)slot * ntr + t];
            const double ld = loads[((int64_t)t * ma.n2 + A) * D + c];
            yu.x -= P.x * ld;
            yu.y -= P.y * ld;
          }
        }
      }
      y.at(slot)[A * D + c] = yu;
    }
    const double2 ps = sum_components<D>(ap);
    if (ok && A < ma.nv && c == 0) {
      double2 yp = cscale(ps, sc);
      if (MODE == SPMV_RESID) yp = csub(f.at(slot)[D * ma.n2 + A], yp);
      if (MODE == SPMV_RHS) yp = make_double2(-yp.x, -yp.y);
      y.at(slot)[D * ma.n2 + A] = yp;
    }
  }
}

// Chebyshev recurrence scalars for step i >= 1 on [lmax/ratio, lmax]:
// rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1}); returns rho_{i-1}, rho_i, delta.
__device__ __forceinline__ void cheb_coef(double lmax, double ratio, int i, double& rprev, double& rcur,
                                          double& delta, double& theta) {
  const double lmin = lmax / ratio;
  theta = 0.5 * (lmax + lmin);
  delta = 0.5 * (lmax - lmin);
  const double sigma = theta / delta;
  double r = 1.0 / sigma, rp = r;
  for (int k = 1; k <= i; ++k) {
    rp = r;
    r = 1.0 / (2.0 * sigma - r);
  }
  rprev = rp;
  rcur = r;
}

// Velocity block, first Chebyshev step: t = insc*v_u - G zhat_p on free rows;
// r = t; d0 = diag^-1 t / theta; z_u = d0.
template <int D>
__global__ void __launch_bounds__(256) k_vinit(MeshArgs ma, Batch b, LaneMap lm, VArg v, VArg z, VArg vt,
                                               double ratio) {
  const Lane L = lane_of(lm, ma.n2);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.p0 + it * lm.Geff;
    if (!(L.rowok && p < lm.G)) continue;
    const int si = p / D, c = p % D;
    const int slot = b.act[si];
    const int64_t A = L.row, DN = D * ma.n2;
    double2* __restrict__ r = vt.at(slot);
    double2* __restrict__ d0 = r + DN;
    double2* __restrict__ zs = z.at(slot);
    const int64_t k = A * D + c;
    if (ma.dmask[A] != 0) {
      r[k] = d0[k] = zs[k] = make_double2(0.0, 0.0);
      continue;
    }
    const double sc = in_scale(b, slot);
    double2 t = cscale(v.at(slot)[k], sc);
    const int nvr = ma.nvc[A];
    const int64_t o21 = ma.rowptr21[A], j0 = ma.rowptr[A];
    const double2* __restrict__ zp = zs + DN;
    for (int jj = 0; jj < nvr; ++jj) {
      const double g = ma.G[(int64_t)c * ma.nnz21 + o21 + jj];
      const double2 pv = zp[ma.col[j0 + jj]];
      t.x -= g * pv.x;
      t.y -= g * pv.y;
    }
    const double lmax = b.lv[slot];
    const double theta = 0.5 * lmax * (1.0 + 1.0 / ratio);
    const double dinv = 1.0 / (ma.mu * ma.Kd[A] + fabs(b.omega[slot]) * ma.rho * ma.Md[A]);
    const double2 dd = cscale(t, dinv / theta);
    r[k] = t;
    d0[k] = dd;
    zs[k] = dd;
  }
}

// Velocity block, Chebyshev step i: r -= A_r d_old; d_new = a d_old + b diag^-1 r; z += d_new.
template <int D>
__global__ void __launch_bounds__(256) k_vstep(MeshArgs ma, Batch b, LaneMap lm, VArg z, VArg vt, double ratio,
                                               int step) {
  const Lane L = lane_of(lm, ma.n2);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.p0 + it * lm.Geff;
    if (!(L.rowok && p < lm.G)) continue;
    const int si = p / D, c = p % D;
    const int slot = b.act[si];
    const int64_t A = L.row, DN = D * ma.n2;
    double2* __restrict__ r = vt.at(slot);
    const double2* __restrict__ dold = r + ((step & 1) ? DN : 2 * DN);
    double2* __restrict__ dnew = r + ((step & 1) ? 2 * DN : DN);
    const int64_t k = A * D + c;
    if (ma.dmask[A] != 0) {
      dnew[k] = make_double2(0.0, 0.0);
      continue;
    }
    const double wr = fabs(b.omega[slot]) * ma.rho;
    double2 q = make_double2(0.0, 0.0);
    for (int64_t j = ma.rowptr[A]; j < ma.rowptr[A + 1]; ++j) {
      const double a = ma.mu * ma.Ks[j] + wr * ma.M[j];
      const double2 dv = dold[(int64_t)ma.col[j] * D + c];
      q.x += a * dv.x;
      q.y += a * dv.y;
    }
    double rp, rc, delta, theta;
    cheb_coef(b.lv[slot], ratio, step, rp, rc, delta, theta);
    const double dinv = 1.0 / (ma.mu * ma.Kd[A] + wr * ma.Md[A]);
    const double2 rn = csub(r[k], q);
    const double2 dk = dold[k];
    const double ca = rc * rp, cb = 2.0 * rc / delta * dinv;
    const double2 dn = make_double2(ca * dk.x + cb * rn.x, ca * dk.y + cb * rn.y);
    r[k] = rn;
    dnew[k] = dn;
    double2* __restrict__ zs = z.at(slot);
    zs[k] = cadd(zs[k], dn);
  }
}

// Pressure block, first step (elementwise over vertices): r = insc*v_p,
// d0 = diag(L)^-1 r / theta, x = d0; with one step the Schur block is final:
// zhat_p = -(mu Mp^-1 v_p + j w rho x).
__global__ void k_pinit(MeshArgs ma, int D, Batch b, VArg v, VArg z, VArg pt, double ratio, int kp) {
  const int64_t vv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vv >= ma.nv) return;
  const int slot = b.act[blockIdx.y];
  const int64_t DN = D * ma.n2, nv = ma.nv;
  const double sc = in_scale(b, slot);
  const double2 vp = cscale(v.at(slot)[DN + vv], sc);
  double2* t = pt.at(slot);
  double2 *rp = t + DN, *d0 = rp + nv, *xp = rp + 3 * nv;
  const double theta = 0.5 * ma.lpmax * (1.0 + 1.0 / ratio);
  const double2 dd = cscale(vp, ma.lpdinv[vv] / theta);
  rp[vv] = vp;
  d0[vv] = dd;
  xp[vv] = dd;
  if (kp == 1) {
    const double wr = b.omega[slot] * ma.rho, im = ma.mu / ma.Mp[vv];
    z.at(slot)[DN + vv] = make_double2(-(im * vp.x - wr * dd.y), -(im * vp.y + wr * dd.x));
  }
}

// Pressure Laplacian, first half: t = diag(M)^-1 G_F d_old (zero on Dirichlet rows).
template <int D>
__global__ void __launch_bounds__(256) k_lp1(MeshArgs ma, Batch b, LaneMap lm, VArg pt, int step) {
  const Lane L = lane_of(lm, ma.n2);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.p0 + it * lm.Geff;
    if (!(L.rowok && p < lm.G)) continue;
    const int si = p / D, c = p % D;
    const int slot = b.act[si];
    const int64_t A = L.row, DN = D * ma.n2, nv = ma.nv;
    double2* t = pt.at(slot);
    const double2* __restrict__ dold = t + DN + ((step & 1) ? nv : 2 * nv);
    double2 acc = make_double2(0.0, 0.0);
    if (ma.dmask[A] == 0) {
      const int nvr = ma.nvc[A];
      const int64_t o21 = ma.rowptr21[A], j0 = ma.rowptr[A];
      for (int jj = 0; jj < nvr; ++jj) {
        const double g = ma.G[(int64_t)c * ma.nnz21 + o21 + jj];
        const double2 pv = dold[ma.col[j0 + jj]];
        acc.x += g * pv.x;
        acc.y += g * pv.y;
      }
      acc = cscale(acc, 1.0 / ma.Md[A]);
    }
    t[A * D + c] = acc;
  }
}

// Pressure Laplacian, second half and Chebyshev step on the vertex rows:
// q = G^T t; r -= q; d_new = a d_old + b diag(L)^-1 r; x += d_new; on the last
// step zhat_p = -(mu Mp^-1 v_p + j w rho x).
template <int D>
__global__ void __launch_bounds__(256) k_lp2(MeshArgs ma, Batch b, LaneMap lm, VArg v, VArg z, VArg pt,
                                             double ratio, int step, int last) {
  const Lane L = lane_of(lm, ma.nv);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.p0 + it * lm.Geff;
    const bool ok = L.rowok && p < lm.G;
    const int si = p / D, c = p % D;
    const int64_t A = L.row;
    int slot = 0;
    double2 q = make_double2(0.0, 0.0);
    if (ok) {
      slot = b.act[si];
      const double2* __restrict__ t = pt.at(slot);
      for (int64_t j = ma.rowptr[A]; j < ma.rowptr[A + 1]; ++j) {
        const double g = ma.Gt[(int64_t)c * ma.nnzv + j];
        const double2 tv = t[(int64_t)ma.col[j] * D + c];
        q.x += g * tv.x;
        q.y += g * tv.y;
      }
    }
    q = sum_components<D>(q);
    if (ok && c == 0) {
      const int64_t DN = D * ma.n2, nv = ma.nv;
      double2* t = pt.at(slot);
      double2 *rp = t + DN, *xp = rp + 3 * nv;
      const double2* dold = rp + ((step & 1) ? nv : 2 * nv);
      double2* dnew = rp + ((step & 1) ? 2 * nv : nv);
      double rpv, rc, delta, theta;
      cheb_coef(ma.lpmax, ratio, step, rpv, rc, delta, theta);
      const double2 rn = csub(rp[A], q);
      const double ca = rc * rpv, cb = 2.0 * rc / delta * ma.lpdinv[A];
      const double2 dk = dold[A];
      const double2 dn = make_double2(ca * dk.x + cb * rn.x, ca * dk.y + cb * rn.y);
      const double2 xn = cadd(xp[A], dn);
      rp[A] = rn;
      dnew[A] = dn;
      xp[A] = xn;
      if (last) {
        const double sc = in_scale(b, slot);
        const double2 vp = cscale(v.at(slot)[DN + A], sc);
        const double wr = b.omega[slot] * ma.rho, im = ma.mu / ma.Mp[A];
        z.at(slot)[DN + A] = make_double2(-(im * vp.x - wr * xn.y), -(im * vp.y + wr * xn.x));
      }
    }
  }
}

// Gershgorin bound of diag^-1 (mu Ks + |w| rho M) over the free rows (free columns).
__global__ void k_vbound(MeshArgs ma, Batch b, unsigned long long* __restrict__ out) {
  __shared__ double sh[256];
  const int slot = b.act[blockIdx.y];
  const double wr = fabs(b.omega[slot]) * ma.rho;
  double mx = 0.0;
  for (int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; A < ma.n2;
       A += (int64_t)gridDim.x * blockDim.x) {
    if (ma.dmask[A] != 0) continue;
    double s = 0.0;
    for (int64_t j = ma.rowptr[A]; j < ma.rowptr[A + 1]; ++j)
      if (ma.dmask[ma.col[j]] == 0) s += fabs(ma.mu * ma.Ks[j] + wr * ma.M[j]);
    mx = fmax(mx, s / (ma.mu * ma.Kd[A] + wr * ma.Md[A]));
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&out[slot], (unsigned long long)__double_as_longlong(sh[0]));
}

inline unsigned row_blocks(int64_t nrows, const LaneMap& lm) {
  const int64_t per = 4 * (int64_t)lm.R;
  return (unsigned)((nrows + per - 1) / per);
}

template <int D>
void full_launch(const MeshArgs& ma, const Batch& b, VArg x, VArg y, int mode, bool mask, VArg f,
                 const double* loads, int ntr, const double2* trac, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nb = row_blocks(ma.n2, lm);
  if (mode == SPMV_APPLY && mask)
    k_full<D, SPMV_APPLY, true><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else if (mode == SPMV_APPLY)
    k_full<D, SPMV_APPLY, false><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else if (mode == SPMV_RESID)
    k_full<D, SPMV_RESID, true><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else
    k_full<D, SPMV_RHS, false><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  launch_check(s);
}

template <int D>
void precond_launch(const MeshArgs& ma, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nbu = row_blocks(ma.n2, lm), nbp = row_blocks(ma.nv, lm);
  dim3 gp((unsigned)((ma.nv + 255) / 256), (unsigned)b.nact);
  k_pinit<<<gp, 256, 0, s>>>(ma, D, b, v, z, pa.pt, pa.ratio, pa.kp);
  for (int i = 1; i < pa.kp; ++i) {
    k_lp1<D><<<nbu, 256, 0, s>>>(ma, b, lm, pa.pt, i);
    k_lp2<D><<<nbp, 256, 0, s>>>(ma, b, lm, v, z, pa.pt, pa.ratio, i, i == pa.kp - 1);
  }
  k_vinit<D><<<nbu, 256, 0, s>>>(ma, b, lm, v, z, pa.vt, pa.ratio);
  for (int i = 1; i < pa.kv; ++i) k_vstep<D><<<nbu, 256, 0, s>>>(ma, b, lm, z, pa.vt, pa.ratio, i);
  launch_check(s);
}

}  // namespace

void spmv_full(scvs_mesh m, const Batch& b, VArg x, VArg y, int mode, bool maskcol, VArg f, const double2* trac,
               hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  const int ntr = (int)m->traction_tags.size();
  if (m->dim == 2)
    full_launch<2>(ma, b, x, y, mode, maskcol, f, m->loads, ntr, trac, s);
  else
    full_launch<3>(ma, b, x, y, mode, maskcol, f, m->loads, ntr, trac, s);
}

void precond_apply(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  if (m->dim == 2)
    precond_launch<2>(ma, b, pa, v, z, s);
  else
    precond_launch<3>(ma, b, pa, v, z, s);
}

void velocity_bounds(scvs_mesh m, const Batch& b, double* lv_out, hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  dim3 g(256, (unsigned)b.nact);
  k_vbound<<<g, 256, 0, s>>>(ma, b, reinterpret_cast<unsigned long long*>(lv_out));
  launch_check(s);
}

}  // namespace scvs

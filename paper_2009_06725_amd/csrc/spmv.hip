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
#include "rowmap.hpp"

namespace scvs {
namespace {

struct MeshArgs {
  int64_t n2, nv, nnz21, nnzv, nnz, nnzl;
  const int64_t *rowptr, *rowptr21;
  const int32_t *col, *nvc, *dmask;
  const double *Ks, *M, *G, *Gt, *Kd, *Md, *Mp, *lpdinv;
  const float *Ks32, *M32, *G32, *Gt32, *Kd32, *Md32;
  const int64_t* lp_ptr;
  const int32_t* lp_col;
  const double* lp_val;
  const float* lp_val32;
  double mu, rho, lpmax;
};

MeshArgs mesh_args(scvs_mesh m) {
  MeshArgs a;
  a.n2 = m->n2;
  a.nv = m->nv;
  a.nnz21 = m->nnz21;
  a.nnzv = m->nnzv;
  a.nnz = m->nnz;
  a.nnzl = m->nnzl;
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
  a.Ks32 = m->Ks32;
  a.M32 = m->M32;
  a.G32 = m->G32;
  a.Gt32 = m->Gt32;
  a.Kd32 = m->Kd32;
  a.Md32 = m->Md32;
  a.lpdinv = m->lpdinv;
  a.lp_ptr = m->lp_ptr;
  a.lp_col = m->lp_col;
  a.lp_val = m->lp_val;
  a.lp_val32 = m->lp_val32;
  a.mu = m->mu;
  a.rho = m->rho;
  a.lpmax = m->lp_lmax;
  return a;
}

// Matrix values and complex vector element type per working precision.
template <class R>
struct Prec;
template <>
struct Prec<double> {
  using C = double2;
  using V = VArg;
  __device__ static const double* Ks(const MeshArgs& a) { return a.Ks; }
  __device__ static const double* M(const MeshArgs& a) { return a.M; }
  __device__ static const double* G(const MeshArgs& a) { return a.G; }
  __device__ static const double* Gt(const MeshArgs& a) { return a.Gt; }
  __device__ static const double* Kd(const MeshArgs& a) { return a.Kd; }
  __device__ static const double* Md(const MeshArgs& a) { return a.Md; }
  __device__ static const double* Lp(const MeshArgs& a) { return a.lp_val; }
};
template <>
struct Prec<float> {
  using C = float2;
  using V = VArg32;
  __device__ static const float* Ks(const MeshArgs& a) { return a.Ks32; }
  __device__ static const float* M(const MeshArgs& a) { return a.M32; }
  __device__ static const float* G(const MeshArgs& a) { return a.G32; }
  __device__ static const float* Gt(const MeshArgs& a) { return a.Gt32; }
  __device__ static const float* Kd(const MeshArgs& a) { return a.Kd32; }
  __device__ static const float* Md(const MeshArgs& a) { return a.Md32; }
  __device__ static const float* Lp(const MeshArgs& a) { return a.lp_val32; }
};

template <class C>
__device__ __forceinline__ C czero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

__device__ __forceinline__ double in_scale(const Batch& b, int slot) {
  return b.insc ? b.insc[(int64_t)slot * b.insc_st + b.insc_idx] : 1.0;
}

// Sum over the D lanes of one system (lanes p = s*D + c are adjacent).
template <int D, class C>
__device__ __forceinline__ C sum_components(C v) {
  C r = v;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    r.x += __shfl_down(v.x, k, 64);
    r.y += __shfl_down(v.y, k, 64);
  }
  return r;
}

// Walk slots [j0, j1) of an S2 row: au += (mu Ks + (ar + j ai) M) x[col] (when
// wantK) and ap += Gt^c x[col] (when wantGt), where the lane's value of node col
// sits at xs[col * xst + xoff] (system-major: xst = D, xoff = c; interleaved
// temporaries: xst = pairs per node, xoff = pair). Every lane of the W-lane row
// group calls this together: the group first loads W slots of (col, Ks, M)
// lane-parallel (coalesced), then broadcasts them by shuffles and issues eight
// independent gathers at a time. With MASK, Dirichlet columns are skipped.
template <int D, bool MASK, class R>
__device__ __forceinline__ void row_acc(const MeshArgs& ma, int W, int li, int64_t j0, int64_t j1,
                                        const typename Prec<R>::C* __restrict__ xs, int64_t xst, int xoff, int c,
                                        bool pairok, R ar, R ai,
                                        bool wantK, bool wantGt, typename Prec<R>::C& au,
                                        typename Prec<R>::C& ap) {
  using C = typename Prec<R>::C;
  constexpr int U = 8;
  const R* __restrict__ Ks = Prec<R>::Ks(ma);
  const R* __restrict__ Mv = Prec<R>::M(ma);
  const R* __restrict__ Gt = Prec<R>::Gt(ma);
  const R mu = (R)ma.mu;
  for (int64_t jb = j0; jb < j1; jb += W) {
    const int n = (int)min((int64_t)W, j1 - jb);
    int32_t mc = 0;
    R mk = 0, mm = 0;
    if (li < n) {
      mc = ma.col[jb + li];
      mk = Ks[jb + li];
      mm = Mv[jb + li];
      if (MASK && ma.dmask[mc] != 0) mc = -1;
    }
    for (int t = 0; t < n; t += U) {
      int32_t B[U];
      R k[U], m[U];
      C xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        B[u] = __shfl(mc, t + u < n ? t + u : 0, W);
        k[u] = __shfl(mk, t + u < n ? t + u : 0, W);
        m[u] = __shfl(mm, t + u < n ? t + u : 0, W);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        xv[u] = (pairok && t + u < n && B[u] >= 0) ? xs[(int64_t)B[u] * xst + xoff] : czero<C>();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (wantK) {
          const R kr = mu * k[u] + ar * m[u], ki = ai * m[u];
          au.x += kr * xv[u].x - ki * xv[u].y;
          au.y += kr * xv[u].y + ki * xv[u].x;
        }
        if (wantGt && pairok && t + u < n) {
          const R g = Gt[(int64_t)c * ma.nnzv + jb + t + u];
          ap.x += g * xv[u].x;
          ap.y += g * xv[u].y;
        }
      }
    }
  }
}

// acc += s * sum_{jj < nvc} G^c[row prefix] p[col] over the vertex-column prefix of a row
// (G in precision R, pressure values of complex type P at p[col * pst + poff],
// accumulation in R).
template <int D, class R, class P>
__device__ __forceinline__ void g_acc(const MeshArgs& ma, int64_t A, int64_t j0, const P* __restrict__ p,
                                      int64_t pst, int poff, int c, R s, typename Prec<R>::C& acc) {
  const int nvr = ma.nvc[A];
  const R* __restrict__ Gc = Prec<R>::G(ma) + (int64_t)c * ma.nnz21 + ma.rowptr21[A];
  const int32_t* __restrict__ cl = ma.col + j0;
  int jj = 0;
  for (; jj + 4 <= nvr; jj += 4) {
    int32_t B[4];
    R g[4];
    P pv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) B[u] = cl[jj + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      g[u] = Gc[jj + u];
      pv[u] = p[(int64_t)B[u] * pst + poff];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc.x += s * g[u] * (R)pv[u].x;
      acc.y += s * g[u] * (R)pv[u].y;
    }
  }
  for (; jj < nvr; ++jj) {
    const P pv = p[(int64_t)cl[jj] * pst + poff];
    acc.x += s * Gc[jj] * (R)pv.x;
    acc.y += s * Gc[jj] * (R)pv.y;
  }
}

// With IL the input is the interleaved vector xil written by the preconditioner inside a
// cycle: velocity pair p of node A at xil[A*G + p], pressure of system si at vertex v at
// xil[n2*G + v*nact + si] (G = nact*D pairs); x is then unused.
template <int D, int MODE, bool MASK, class R, bool IL = false, class YT = double2>
__global__ void __launch_bounds__(256) k_full(MeshArgs ma, Batch b, LaneMap lm, typename Prec<R>::V x, SV<YT> y,
                                              VArg f, const double* __restrict__ loads, int ntr,
                                              const double2* __restrict__ trac,
                                              const typename Prec<R>::C* __restrict__ xil = nullptr) {
  using C = typename Prec<R>::C;
  const Lane L = lane_of(lm, ma.n2);
  if (!L.rowok) return;  // uniform over the row group
  const int64_t A = L.row;
  const int32_t dm = ma.dmask[A];
  const bool isv = A < ma.nv;
  const int64_t j0 = ma.rowptr[A], j1 = ma.rowptr[A + 1];
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    const bool ok = L.pairok0 && p < lm.G;
    const int si = ok ? p / D : 0, c = ok ? p % D : 0;
    const int slot = b.act[si];
    const double sc = in_scale(b, slot);
    const C* __restrict__ xs = IL ? xil : x.at(slot);
    const int64_t xst = IL ? lm.G : D;
    const int xo = IL ? p : c;
    const R wr = (R)(b.omega[slot] * ma.rho);
    C au = czero<C>(), ap = czero<C>();
    if (dm == 0 || isv)
      row_acc<D, MASK, R>(ma, lm.W, L.li, j0, j1, xs, xst, xo, c, ok, (R)0, wr, dm == 0, isv, au, ap);
    if (ok) {
      if (dm == 0) {
        if (IL)
          g_acc<D, R, C>(ma, A, j0, xil + ma.n2 * lm.G, b.nact, si, c, (R)1, au);
        else
          g_acc<D, R, C>(ma, A, j0, xs + D * ma.n2, 1, 0, c, (R)1, au);
      }
      double2 yu;
      if (dm != 0) {
        const C xv = xs[A * xst + xo];
        yu = make_double2(sc * (double)xv.x, sc * (double)xv.y);
        if (MODE == SPMV_RESID) yu = csub(f.at(slot)[A * D + c], yu);
      } else {
        const double2 a = make_double2(sc * (double)au.x, sc * (double)au.y);
        if (MODE == SPMV_APPLY) {
          yu = a;
        } else if (MODE == SPMV_RESID) {
          yu = csub(f.at(slot)[A * D + c], a);
        } else {
          yu = make_double2(-a.x, -a.y);
          for (int t = 0; t < ntr; ++t) {
            const double2 P = trac[(int64_t)slot * ntr + t];
            const double ld = loads[((int64_t)t * ma.n2 + A) * D + c];
            yu.x -= P.x * ld;
            yu.y -= P.y * ld;
          }
        }
      }
      y.at(slot)[A * D + c] = cvt2<YT>(yu);
    }
    if (isv) {
      const C ps = sum_components<D, C>(ap);
      if (ok && c == 0) {
        double2 yp = make_double2(sc * (double)ps.x, sc * (double)ps.y);
        if (MODE != SPMV_RHS && b.pen != 0.0) {  // penalized continuity block -pen Mp p
          const C xp = IL ? xil[ma.n2 * lm.G + A * b.nact + si] : xs[D * ma.n2 + A];
          const double w = b.pen * ma.Mp[A] * sc;
          yp.x -= w * (double)xp.x;
          yp.y -= w * (double)xp.y;
        }
        if (MODE == SPMV_RESID) yp = csub(f.at(slot)[D * ma.n2 + A], yp);
        if (MODE == SPMV_RHS) yp = make_double2(-yp.x, -yp.y);
        y.at(slot)[D * ma.n2 + A] = cvt2<YT>(yp);
      }
    }
  }
}

// S2 in sliced rows for the FP32 operator product (layout of struct Sell).
struct S2SellArgs {
  int64_t nslot, vslots;      // slots; slots of the vertex rows (the first slices)
  const int64_t *off, *goff;  // entries per slice of S2 and of the vertex-column prefix
  const int32_t* row;
  const int32_t* col;
  const float *K, *M;
  const float* G;   // [goff[end]][D]: G^c on the vertex-column prefix of each row
  const float* Gt;  // [off[vslots / SELL_C]][D]: G^T^c on the vertex rows' entries
};

// k_full (operator product y = A x, FP32 values, interleaved input xil) in sliced
// rows: one lane per (row, system) holds that system's D momentum sums, and on a
// vertex row also its divergence sum; entry t of the wavefront's rows is one
// contiguous load of columns and of each value array. Same arithmetic and outputs as
// k_full<D, SPMV_APPLY, false, float, true, YT>.
template <int D, class YT>
__global__ void __launch_bounds__(256) k_full_sell(MeshArgs ma, S2SellArgs sa, Batch b, int W, int RW,
                                                   const float2* __restrict__ xil, SV<YT> y) {
  constexpr int U = 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * RW + lane / W;
  if (q >= sa.nslot) return;
  const int32_t A = sa.row[q];
  if (A < 0) return;
  const int64_t sl = q / SELL_C, r = q % SELL_C;
  const int64_t e0 = sa.off[sl] + r, g0 = sa.goff[sl] + r;
  const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
  const int glen = (int)((sa.goff[sl + 1] - sa.goff[sl]) / SELL_C);
  const bool isv = q < sa.vslots;
  const int32_t dm = ma.dmask[A];
  const int nvr = ma.nvc[A];
  const int G = b.nact * D;
  const float2* __restrict__ pil = xil + ma.n2 * G;  // pressures: [nv][nact]
  const float mu = (float)ma.mu;
  for (int si = lane & (W - 1); si < b.nact; si += W) {
    const int slot = b.act[si];
    const double sc = in_scale(b, slot);
    const float wr = (float)(b.omega[slot] * ma.rho);
    const float2* __restrict__ xs = xil + si * D;
    float2 au[D], ap = make_float2(0.f, 0.f);
#pragma unroll
    for (int d = 0; d < D; ++d) au[d] = make_float2(0.f, 0.f);
    if (dm == 0 || isv) {
      for (int t = 0; t < len; t += U) {
        int32_t c[U];
        float k[U], m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool v = t + u < len;
          const int64_t e = e0 + (int64_t)(t + u) * SELL_C;
          c[u] = v ? sa.col[e] : -1;
          k[u] = v ? sa.K[e] : 0.f;
          m[u] = v ? sa.M[e] : 0.f;
        }
        float2 xv[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int d = 0; d < D; ++d) xv[u][d] = c[u] >= 0 ? xs[(int64_t)c[u] * G + d] : make_float2(0.f, 0.f);
        if (dm == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const float kr = mu * k[u], ki = wr * m[u];
#pragma unroll
            for (int d = 0; d < D; ++d) {
              au[d].x += kr * xv[u][d].x - ki * xv[u][d].y;
              au[d].y += kr * xv[u][d].y + ki * xv[u][d].x;
            }
          }
          if (t < glen) {  // G p over the vertex-column prefix
#pragma unroll
            for (int u = 0; u < U; ++u) {
              if (t + u < nvr) {
                const int64_t ge = (g0 + (int64_t)(t + u) * SELL_C) * D;
                const float2 pv = pil[(int64_t)c[u] * b.nact + si];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                  const float g = sa.G[ge + d];
                  au[d].x += g * pv.x;
                  au[d].y += g * pv.y;
                }
              }
            }
          }
        }
        if (isv) {  // divergence row: sum_c G^T^c x_c
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (t + u < len) {
              const int64_t e = (e0 + (int64_t)(t + u) * SELL_C) * D;
#pragma unroll
              for (int d = 0; d < D; ++d) {
                const float g = sa.Gt[e + d];
                ap.x += g * xv[u][d].x;
                ap.y += g * xv[u][d].y;
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double2 yu;
      if (dm != 0) {
        const float2 xv = xs[(int64_t)A * G + d];
        yu = make_double2(sc * (double)xv.x, sc * (double)xv.y);
      } else {
        yu = make_double2(sc * (double)au[d].x, sc * (double)au[d].y);
      }
      y.at(slot)[(int64_t)A * D + d] = cvt2<YT>(yu);
    }
    if (isv) {
      double2 yp = make_double2(sc * (double)ap.x, sc * (double)ap.y);
      if (b.pen != 0.0) {  // penalized continuity block -pen Mp p
        const float2 xp = pil[(int64_t)A * b.nact + si];
        const double w = b.pen * ma.Mp[A] * sc;
        yp.x -= w * (double)xp.x;
        yp.y -= w * (double)xp.y;
      }
      y.at(slot)[(int64_t)D * ma.n2 + A] = cvt2<YT>(yp);
    }
  }
}

// Value of lane U of each group of four lanes (DPP quad broadcast).
template <int U>
__device__ __forceinline__ int qbc(int v) {
  return __builtin_amdgcn_mov_dpp(v, U * 0x55, 0xF, 0xF, false);
}
template <int U>
__device__ __forceinline__ float qbc(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), U * 0x55, 0xF, 0xF, false));
}

// k_full_sell for rows of 6 or 8 (system, component) pairs: four lanes per row, each
// with two pairs gathered by one 16-byte load; the four lanes load four entries'
// (column, Ks, M) at once and share them by quad broadcasts. A vertex row's divergence
// sums are per pair and are summed per system over the four lanes. Same products as
// k_full_sell; outputs per pair and, on vertex rows, per system.
template <int D, class YT>
__global__ void __launch_bounds__(256) k_full_sell4(MeshArgs ma, S2SellArgs sa, Batch b,
                                                    const float2* __restrict__ xil, SV<YT> y) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * 16 + lane / 4;
  if (q >= sa.nslot) return;
  const int32_t A = sa.row[q];
  if (A < 0) return;  // uniform over the four lanes of the row
  const int64_t sl = q / SELL_C, r = q % SELL_C;
  const int64_t e0 = sa.off[sl] + r, g0 = sa.goff[sl] + r;
  const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
  const int glen = (int)((sa.goff[sl + 1] - sa.goff[sl]) / SELL_C);
  const bool isv = q < sa.vslots;  // uniform over a slice
  const int32_t dm = ma.dmask[A];
  const int nvr = ma.nvc[A];
  const int G = b.nact * D, li = lane & 3, p0 = 2 * li;
  const bool act = p0 < G;
  const int s0 = act ? p0 / D : 0, s1 = act ? (p0 + 1) / D : 0;
  const int d0 = p0 % D, d1 = (p0 + 1) % D;
  const int slot0 = b.act[s0], slot1 = b.act[s1];
  const float mu = (float)ma.mu;
  const float w0 = (float)(b.omega[slot0] * ma.rho), w1 = (float)(b.omega[slot1] * ma.rho);
  const float2* __restrict__ pil = xil + ma.n2 * G;  // pressures: [nv][nact]
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  float2 q0 = make_float2(0.f, 0.f), q1 = make_float2(0.f, 0.f);  // divergence parts per pair
  if (dm == 0 || isv) {
    for (int t = 0; t < len; t += 4) {
      const bool vl = t + li < len;
      const int64_t el = e0 + (int64_t)(t + li) * SELL_C;
      const int32_t cl = vl ? sa.col[el] : -1;
      const float kl = vl ? sa.K[el] : 0.f, ml = vl ? sa.M[el] : 0.f;
      int32_t c[4];
      float k[4], m[4];
      c[0] = qbc<0>(cl); c[1] = qbc<1>(cl); c[2] = qbc<2>(cl); c[3] = qbc<3>(cl);
      k[0] = qbc<0>(kl); k[1] = qbc<1>(kl); k[2] = qbc<2>(kl); k[3] = qbc<3>(kl);
      m[0] = qbc<0>(ml); m[1] = qbc<1>(ml); m[2] = qbc<2>(ml); m[3] = qbc<3>(ml);
      float4 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        xv[u] = (act && c[u] >= 0) ? *reinterpret_cast<const float4*>(xil + (int64_t)c[u] * G + p0)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
      if (dm == 0 && act) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float kr = mu * k[u], ki0 = w0 * m[u], ki1 = w1 * m[u];
          a0.x += kr * xv[u].x - ki0 * xv[u].y;
          a0.y += kr * xv[u].y + ki0 * xv[u].x;
          a1.x += kr * xv[u].z - ki1 * xv[u].w;
          a1.y += kr * xv[u].w + ki1 * xv[u].z;
        }
        if (t < glen) {  // G p over the vertex-column prefix
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (t + u < nvr) {
              const int64_t ge = (g0 + (int64_t)(t + u) * SELL_C) * D;
              const float2 pv0 = pil[(int64_t)c[u] * b.nact + s0];
              const float2 pv1 = pil[(int64_t)c[u] * b.nact + s1];
              const float g0v = sa.G[ge + d0], g1v = sa.G[ge + d1];
              a0.x += g0v * pv0.x;
              a0.y += g0v * pv0.y;
              a1.x += g1v * pv1.x;
              a1.y += g1v * pv1.y;
            }
          }
        }
      }
      if (isv && act) {  // divergence row: G^T^d x_(s, d) per pair
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (c[u] >= 0) {
            const int64_t e = (e0 + (int64_t)(t + u) * SELL_C) * D;
            const float g0v = sa.Gt[e + d0], g1v = sa.Gt[e + d1];
            q0.x += g0v * xv[u].x;
            q0.y += g0v * xv[u].y;
            q1.x += g1v * xv[u].z;
            q1.y += g1v * xv[u].w;
          }
        }
      }
    }
  }
  if (act) {
    const int64_t o = (int64_t)A * G + p0;
    double2 y0, y1;
    const double sc0 = in_scale(b, slot0), sc1 = in_scale(b, slot1);
    if (dm != 0) {
      const float4 xa = *reinterpret_cast<const float4*>(xil + o);
      y0 = make_double2(sc0 * (double)xa.x, sc0 * (double)xa.y);
      y1 = make_double2(sc1 * (double)xa.z, sc1 * (double)xa.w);
    } else {
      y0 = make_double2(sc0 * (double)a0.x, sc0 * (double)a0.y);
      y1 = make_double2(sc1 * (double)a1.x, sc1 * (double)a1.y);
    }
    y.at(slot0)[(int64_t)A * D + d0] = cvt2<YT>(y0);
    y.at(slot1)[(int64_t)A * D + d1] = cvt2<YT>(y1);
  }
  if (isv) {
    // per system s: the sum over its D pairs, in pair order, gathered from the quad
    for (int si = 0; si < b.nact; ++si) {
      float2 part = make_float2(0.f, 0.f);
      if (act && s0 == si) { part.x += q0.x; part.y += q0.y; }
      if (act && s1 == si) { part.x += q1.x; part.y += q1.y; }
      float px[4], py[4];
      px[0] = qbc<0>(part.x); px[1] = qbc<1>(part.x); px[2] = qbc<2>(part.x); px[3] = qbc<3>(part.x);
      py[0] = qbc<0>(part.y); py[1] = qbc<1>(part.y); py[2] = qbc<2>(part.y); py[3] = qbc<3>(part.y);
      if (li != si) continue;
      const float2 ap = make_float2(((px[0] + px[1]) + px[2]) + px[3], ((py[0] + py[1]) + py[2]) + py[3]);
      const int slot = b.act[si];
      const double sc = in_scale(b, slot);
      double2 yp = make_double2(sc * (double)ap.x, sc * (double)ap.y);
      if (b.pen != 0.0) {  // penalized continuity block -pen Mp p
        const float2 xp = pil[(int64_t)A * b.nact + si];
        const double w = b.pen * ma.Mp[A] * sc;
        yp.x -= w * (double)xp.x;
        yp.y -= w * (double)xp.y;
      }
      y.at(slot)[(int64_t)D * ma.n2 + A] = cvt2<YT>(yp);
    }
  }
}

// Lumped outlets: after the operator kernel, y += s * sc * Z_o(w) (b_o^T x) b_o on the
// free momentum rows of every outlet o, s = +1 for y = A x and -1 for y = f - A x and
// for the right-hand side (where x is the Dirichlet lift and b_o^T x runs over the
// prescribed-inflow unknowns, as the symmetric elimination moves them). One block
// per system: fixed-order block sums for the flows, then the rank-one updates.
struct WkArgs {
  int n;
  const double* par;
  const int64_t* qoff;
  const int32_t* qdof;
  const double* qb;
  int64_t nrow;
  const int64_t* roff;
  const int32_t* rdof;
  const int32_t* rout;
  const double* rb;
};

WkArgs wk_args(scvs_mesh m) {
  return {m->nwk,  m->wk_dpar, m->wk_qoff, m->wk_qdof, m->wk_qb,
          m->wk_nrow, m->wk_roff, m->wk_rdof, m->wk_rout, m->wk_rb};
}

template <int D, class XC, bool IL, class YT>
__global__ void __launch_bounds__(256) k_wk(WkArgs w, Batch b, int mode, SV<XC> x, const XC* __restrict__ xil,
                                            int G, SV<YT> y) {
  __shared__ double2 part[4];
  __shared__ double2 zq[SCVS_WK_MAX];
  const int si = blockIdx.x;
  const int slot = b.act[si];
  const XC* __restrict__ xs = IL ? nullptr : x.at(slot);
  const int half = mode == SPMV_RHS ? 1 : 0;
  for (int o = 0; o < w.n; ++o) {
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t e = w.qoff[2 * o + half] + threadIdx.x; e < w.qoff[2 * o + half + 1]; e += blockDim.x) {
      const int32_t dof = w.qdof[e];
      const XC v = IL ? xil[(int64_t)(dof / D) * G + si * D + dof % D] : xs[dof];
      acc.x += w.qb[e] * (double)v.x;
      acc.y += w.qb[e] * (double)v.y;
    }
    for (int off = 32; off > 0; off >>= 1) {
      acc.x += __shfl_down(acc.x, off);
      acc.y += __shfl_down(acc.y, off);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const double2 q = make_double2(part[0].x + part[1].x + part[2].x + part[3].x,
                                     part[0].y + part[1].y + part[2].y + part[3].y);
      // Z = rp + rd / (1 + j w rd c)
      const double rp = w.par[3 * o], cc = w.par[3 * o + 1], rd = w.par[3 * o + 2];
      const double t = b.omega[slot] * rd * cc, den = 1.0 + t * t;
      const double zr = rp + rd / den, zi = -rd * t / den;
      const double sg = (mode == SPMV_APPLY ? 1.0 : -1.0) * in_scale(b, slot);
      zq[o] = make_double2(sg * (zr * q.x - zi * q.y), sg * (zr * q.y + zi * q.x));
    }
    __syncthreads();
  }
  YT* __restrict__ ys = y.at(slot);
  for (int64_t r = threadIdx.x; r < w.nrow; r += blockDim.x) {
    double2 add = make_double2(0.0, 0.0);
    for (int64_t e = w.roff[r]; e < w.roff[r + 1]; ++e) {
      const double2 q = zq[w.rout[e]];
      add.x += q.x * w.rb[e];
      add.y += q.y * w.rb[e];
    }
    const int32_t dof = w.rdof[r];
    const YT old = ys[dof];
    ys[dof] = cvt2<YT>(make_double2((double)old.x + add.x, (double)old.y + add.y));
  }
}

template <class XC, bool IL, class YT>
void wk_launch(scvs_mesh m, const Batch& b, int mode, SV<XC> x, const XC* xil, SV<YT> y, hipStream_t s) {
  if (m->nwk == 0 || b.no_lumped || b.nact == 0) return;
  const WkArgs w = wk_args(m);
  const int D = m->dim;
  ProfScope ps(&m->ctx->prof, s, "k_wk", 0.0);
  if (D == 2)
    k_wk<2, XC, IL, YT><<<b.nact, 256, 0, s>>>(w, b, mode, x, xil, b.nact * 2, y);
  else
    k_wk<3, XC, IL, YT><<<b.nact, 256, 0, s>>>(w, b, mode, x, xil, b.nact * 3, y);
  launch_check(s);
}


// Velocity block, Chebyshev polynomial in diag^-1 A_r with A_r = mu Ks + |w| rho M
// (same for every component), in three-term form
//   x_1 = diag^-1 b / theta,
//   x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1}) + (2 rho_k / delta) diag^-1 (b - A_r x_k),
// with b = insc*v_u - G zhat_p. The last iterate is written into z (system-major);
// Dirichlet rows stay zero.
//
// The temporaries b, x_a, x_b, x_c live only inside one application, so they use
// the layout that suits the gathers: pair p = si*D + c of the batch's active list
// (si-th active system, component c) of node A sits at A*G + p (G = pairs), and the
// values that one column contributes to all systems and components are adjacent.
template <class C>
struct ITemps {
  C* base;
  int64_t n2;
  int G;
  __device__ C* arr(int k) const { return base + (int64_t)k * n2 * G; }  // 0: b, 1..3: iterates
  __device__ C* iter(int k) const { return arr(1 + k % 3); }
};

// In FP32 mode the output z is the FP32 vector z32 (velocity part written
// here, pressure part copied from the FP64 Schur-block result zp).
// With zil the result goes to the interleaved vector read by the next operator product
// (layout of k_full's IL input); the pressure part is copied there too.
// With CX (multigrid velocity block) x_1 = D^-1 b / theta uses the complex diagonal
// D = mu Ks_AA + j w rho M_AA of level 0 and the level's bound b.lv.
template <int D, class R, class VI, bool CX = false>
__global__ void __launch_bounds__(256) k_vinit(MeshArgs ma, Batch b, LaneMap lm, SV<VI> v, VArg zp64,
                                               typename Prec<R>::V z, ITemps<typename Prec<R>::C> vt,
                                               double ratio, int kv, typename Prec<R>::C* __restrict__ zil) {
  using C = typename Prec<R>::C;
  const Lane L = lane_of(lm, ma.n2);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    if (!(L.rowok && L.pairok0 && p < lm.G)) continue;
    const int si = p / D, c = p % D;
    const int slot = b.act[si];
    const int64_t A = L.row, DN = D * ma.n2;
    const int64_t k = A * D + c, ki = A * lm.G + p;
    C* __restrict__ bb = vt.arr(0);
    C* __restrict__ x1 = (kv == 1) ? (zil ? zil + ki : z.at(slot) + k) : vt.iter(1) + ki;
    const double2* __restrict__ zp = zp64.at(slot) + DN;
    if ((zil || sizeof(R) == 4) && A < ma.nv && c == 0) {
      const double2 q = zp[A];
      C qq;
      qq.x = (R)q.x;
      qq.y = (R)q.y;
      if (zil)
        zil[ma.n2 * lm.G + A * b.nact + si] = qq;
      else
        z.at(slot)[DN + A] = qq;
    }
    if (ma.dmask[A] != 0) {
      bb[ki] = *x1 = czero<C>();
      continue;
    }
    const double sc = in_scale(b, slot);
    const double2 vv = to_d2(v.at(slot)[k]);
    C t;
    t.x = (R)(sc * vv.x);
    t.y = (R)(sc * vv.y);
    g_acc<D, R, double2>(ma, A, ma.rowptr[A], zp, 1, 0, c, (R)-1, t);
    const double lmax = b.lv[slot];
    const R theta = (R)(0.5 * lmax * (1.0 + 1.0 / ratio));
    bb[ki] = t;
    C xv;
    if (CX) {
      const R dr = (R)ma.mu * Prec<R>::Kd(ma)[A], di = (R)(b.omega[slot] * ma.rho) * Prec<R>::Md(ma)[A];
      const R sc2 = (R)1 / ((dr * dr + di * di) * theta);
      xv.x = (t.x * dr + t.y * di) * sc2;
      xv.y = (t.y * dr - t.x * di) * sc2;
    } else {
      const R dinv = (R)1 / ((R)ma.mu * Prec<R>::Kd(ma)[A] + (R)(fabs(b.omega[slot]) * ma.rho) * Prec<R>::Md(ma)[A]);
      xv.x = t.x * (dinv / theta);
      xv.y = t.y * (dinv / theta);
    }
    *x1 = xv;
  }
}

// k_vinit<D, float, VI, true> (multigrid velocity block, FP32 temporaries, interleaved
// result) in sliced rows: one lane per (row, system) forms b = v_u - G z_p for its D
// components from the G slices and the first smoothing iterate x_1 = D^-1 b / theta
// of level 0, and copies z_p to the interleaved result on a vertex row.
template <int D, class VI>
__global__ void __launch_bounds__(256) k_vinit_sell(MeshArgs ma, S2SellArgs sa, Batch b, int W, int RW, SV<VI> v,
                                                    VArg zp64, ITemps<float2> vt, double ratio,
                                                    float2* __restrict__ zil) {
  constexpr int U = 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * RW + lane / W;
  if (q >= sa.nslot) return;
  const int32_t A = sa.row[q];
  if (A < 0) return;
  const int64_t sl = q / SELL_C, r = q % SELL_C;
  const int64_t e0 = sa.off[sl] + r, g0 = sa.goff[sl] + r;
  const int glen = min((int)((sa.goff[sl + 1] - sa.goff[sl]) / SELL_C), ma.nvc[A]);
  const int G = b.nact * D;
  const int64_t DN = (int64_t)D * ma.n2;
  const bool dir = ma.dmask[A] != 0;
  for (int si = lane & (W - 1); si < b.nact; si += W) {
    const int slot = b.act[si];
    const double2* __restrict__ zp = zp64.at(slot) + DN;
    if (A < ma.nv) {
      const double2 pq = zp[A];
      zil[ma.n2 * G + (int64_t)A * b.nact + si] = make_float2((float)pq.x, (float)pq.y);
    }
    const int64_t o = (int64_t)A * G + si * D;
    float2* __restrict__ bb = vt.arr(0);
    float2* __restrict__ x1 = vt.iter(1);
    if (dir) {
#pragma unroll
      for (int d = 0; d < D; ++d) bb[o + d] = x1[o + d] = make_float2(0.f, 0.f);
      continue;
    }
    const double sc = in_scale(b, slot);
    float2 t[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double2 vv = to_d2(v.at(slot)[(int64_t)A * D + d]);
      t[d] = make_float2((float)(sc * vv.x), (float)(sc * vv.y));
    }
    for (int jt = 0; jt < glen; jt += U) {
      int32_t c[U];
      float2 pv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) c[u] = jt + u < glen ? sa.col[e0 + (int64_t)(jt + u) * SELL_C] : -1;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2 pd = c[u] >= 0 ? zp[c[u]] : make_double2(0.0, 0.0);
        pv[u] = make_float2((float)pd.x, (float)pd.y);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (c[u] < 0) continue;
        const int64_t ge = (g0 + (int64_t)(jt + u) * SELL_C) * D;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const float g = sa.G[ge + d];
          t[d].x += -1.f * g * pv[u].x;
          t[d].y += -1.f * g * pv[u].y;
        }
      }
    }
    const float theta = (float)(0.5 * b.lv[slot] * (1.0 + 1.0 / ratio));
    const float dr = (float)ma.mu * ma.Kd32[A], di = (float)(b.omega[slot] * ma.rho) * ma.Md32[A];
    const float sc2 = 1.f / ((dr * dr + di * di) * theta);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      bb[o + d] = t[d];
      x1[o + d] = make_float2((t[d].x * dr + t[d].y * di) * sc2, (t[d].y * dr - t[d].x * di) * sc2);
    }
  }
}

template <int D, class R>
__global__ void __launch_bounds__(256) k_vstep(MeshArgs ma, Batch b, LaneMap lm, typename Prec<R>::V z,
                                               ITemps<typename Prec<R>::C> vt, double ratio, ChebStep cs, int step,
                                               int last, typename Prec<R>::C* __restrict__ zil) {
  using C = typename Prec<R>::C;
  const Lane L = lane_of(lm, ma.n2);
  if (!L.rowok) return;  // uniform over the row group
  const int64_t A = L.row;
  const bool dir = ma.dmask[A] != 0;
  const int64_t j0 = ma.rowptr[A], j1 = ma.rowptr[A + 1];
  const C* __restrict__ xk = vt.iter(step);
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    const bool ok = L.pairok0 && p < lm.G;
    const int si = ok ? p / D : 0, c = ok ? p % D : 0;
    const int slot = b.act[si];
    const int64_t ki = A * lm.G + p;
    C* __restrict__ xn = last ? (zil ? zil + ki : z.at(slot) + A * D + c) : vt.iter(step + 1) + ki;
    if (dir) {
      if (ok) *xn = czero<C>();
      continue;
    }
    const R wr = (R)(fabs(b.omega[slot]) * ma.rho);
    C q = czero<C>(), unused = czero<C>();
    row_acc<D, false, R>(ma, lm.W, L.li, j0, j1, xk, lm.G, p, c, ok, wr, (R)0, true, false, q, unused);
    if (!ok) continue;
    const double rp = cs.rprev, rc = cs.rcur, delta = 0.5 * b.lv[slot] * (1.0 - 1.0 / ratio);
    const R dinv = (R)1 / ((R)ma.mu * Prec<R>::Kd(ma)[A] + wr * Prec<R>::Md(ma)[A]);
    const C bv = vt.arr(0)[ki], xv = xk[ki];
    const C xo = (step == 1) ? czero<C>() : vt.iter(step - 1)[ki];
    const R ca = (R)(rc * rp), cb = (R)(2.0 * rc / delta) * dinv;
    C o;
    o.x = xv.x + ca * (xv.x - xo.x) + cb * (bv.x - q.x);
    o.y = xv.y + ca * (xv.y - xo.y) + cb * (bv.y - q.y);
    *xn = o;
  }
}

// Pressure block, first step (elementwise over vertices): b = insc*v_p and the first
// Chebyshev iterate x_1 = diag(L)^-1 b / theta; with one step the Schur block is final:
// zhat_p = -(mu Mp^-1 v_p + j w rho x_1). Temps (b, then rotating iterates) are
// interleaved like the velocity ones: system si of the active list at vertex A sits at
// A*G + si.
template <class VI, class R>
__global__ void k_pinit(MeshArgs ma, int D, Batch b, SV<VI> v, VArg z, ITemps<typename Prec<R>::C> pt, double ratio,
                        int kp) {
  using C = typename Prec<R>::C;
  const int64_t vv = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (vv >= ma.nv) return;
  const int si = blockIdx.y;
  const int slot = b.act[si];
  const int64_t DN = D * ma.n2, ki = vv * pt.G + si;
  const double sc = in_scale(b, slot);
  const double2 vp = cscale(to_d2(v.at(slot)[DN + vv]), sc);
  const double theta = 0.5 * ma.lpmax * (1.0 + 1.0 / ratio);
  const double2 dd = cscale(vp, ma.lpdinv[vv] / theta);
  pt.arr(0)[ki] = cvt2<C>(vp);
  pt.iter(1)[ki] = cvt2<C>(dd);
  // without a Laplacian term (w = 0 and no steady pseudo-frequency) the block is final
  // here and the Chebyshev steps skip this system
  const double ws = schur_w(b, slot);
  if (kp <= 1 || ws == 0.0) {
    // kp == 0: the Schur block is the pressure mass alone, zhat_p = -mu Mp^-1 v_p
    const double2 xl = kp == 0 ? make_double2(0.0, 0.0) : dd;
    const double wr = ws * ma.rho, im = ma.mu / ma.Mp[vv];
    z.at(slot)[DN + vv] = make_double2(-(im * vp.x - wr * xl.y), -(im * vp.y + wr * xl.x));
  }
}

// Pressure Laplacian Chebyshev step i on the assembled L, three-term form:
// x_{i+1} = x_i + rho_i rho_{i-1} (x_i - x_{i-1}) + (2 rho_i / delta) diag(L)^-1 (b - L x_i)
// (x_0 = 0); on the last step zhat_p = -(mu Mp^-1 v_p + j w rho x_kp) instead of a store.
// Lanes do not cooperate here, so threads map linearly onto (vertex, system) pairs: every
// lane works, and the systems of one vertex sit in adjacent lanes (coalesced gathers).
template <class VI, class R>
__global__ void __launch_bounds__(256) k_pstep(MeshArgs ma, int D, Batch b, SV<VI> v, VArg z,
                                               ITemps<typename Prec<R>::C> pt, double ratio, ChebStep cs, int step,
                                               int last) {
  using C = typename Prec<R>::C;
  const R* __restrict__ lval = Prec<R>::Lp(ma);
  const int G = pt.G;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ma.nv * G) return;
  const int64_t A = idx / G;
  const int p = (int)(idx - A * G);
  const int slot = b.act[p];
  if (schur_w(b, slot) == 0.0) return;  // Schur block already final (k_pinit)
  const int64_t ki = idx;  // = A * G + p
  const C* __restrict__ xk = pt.iter(step);
  C q = czero<C>();
  const int64_t k0 = ma.lp_ptr[A], k1 = ma.lp_ptr[A + 1];
  int64_t k = k0;
  for (; k + 4 <= k1; k += 4) {
    int32_t u[4];
    R l[4];
    C dv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = ma.lp_col[k + t];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      l[t] = lval[k + t];
      dv[t] = xk[(int64_t)u[t] * G + p];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      q.x += l[t] * dv[t].x;
      q.y += l[t] * dv[t].y;
    }
  }
  for (; k < k1; ++k) {
    const R l = lval[k];
    const C dv = xk[(int64_t)ma.lp_col[k] * G + p];
    q.x += l * dv.x;
    q.y += l * dv.y;
  }
  const double delta = 0.5 * ma.lpmax * (1.0 - 1.0 / ratio);
  const C bv = pt.arr(0)[ki], xv = xk[ki];
  const C xo = step == 1 ? czero<C>() : pt.iter(step - 1)[ki];
  const R ca = (R)(cs.rcur * cs.rprev), cb = (R)(2.0 * cs.rcur / delta * ma.lpdinv[A]);
  C xn;
  xn.x = xv.x + ca * (xv.x - xo.x) + cb * (bv.x - q.x);
  xn.y = xv.y + ca * (xv.y - xo.y) + cb * (bv.y - q.y);
  if (!last) {
    pt.iter(step + 1)[ki] = xn;
  } else {
    // the pressure-mass Schur scaling and the combination stay FP64
    const int64_t DN = D * ma.n2;
    const double sc = in_scale(b, slot);
    const double2 vp = cscale(to_d2(v.at(slot)[DN + A]), sc);
    const double wr = schur_w(b, slot) * ma.rho, im = ma.mu / ma.Mp[A];
    const double2 xd = to_d2(xn);
    z.at(slot)[DN + A] = make_double2(-(im * vp.x - wr * xd.y), -(im * vp.y + wr * xd.x));
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


// Algorithmic bytes of one full-operator launch: every matrix array once
// (S2 col/Ks/M, G on the vertex-column prefix, Gt on vertex rows, row
// pointers, counts and masks) and, per system, x read once and y written once
// (plus f read in residual mode).
double full_bytes(const MeshArgs& ma, int D, int nact, int mode) {
  const double mat = (double)ma.nnz * 20.0 + (double)ma.nnz21 * (4.0 + 8.0 * D) +
                     (double)ma.nnzv * 8.0 * D + (double)ma.n2 * 24.0;
  const double ndof = (double)D * ma.n2 + ma.nv;
  return mat + nact * ndof * 16.0 * (mode == SPMV_RESID ? 3.0 : 2.0);
}

template <int D>
void full_launch(Profiler* prof, const MeshArgs& ma, const Batch& b, VArg x, VArg y, int mode, bool mask, VArg f,
                 const double* loads, int ntr, const double2* trac, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nb = row_blocks(ma.n2, lm);
  const char* nm = mode == SPMV_APPLY ? "k_full_apply" : (mode == SPMV_RESID ? "k_full_resid" : "k_full_rhs");
  ProfScope ps(prof, s, nm, full_bytes(ma, D, b.nact, mode));
  if (mode == SPMV_APPLY && mask)
    k_full<D, SPMV_APPLY, true, double><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else if (mode == SPMV_APPLY)
    k_full<D, SPMV_APPLY, false, double><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else if (mode == SPMV_RESID)
    k_full<D, SPMV_RESID, true, double><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  else
    k_full<D, SPMV_RHS, false, double><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, loads, ntr, trac);
  launch_check(s);
}

template <int D>
void full_launch32(Profiler* prof, const MeshArgs& ma, const Batch& b, VArg32 x, VArg y, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nb = row_blocks(ma.n2, lm);
  // FP32 matrix values (col int32, values float), FP32 input, FP64 output
  const double mat = (double)ma.nnz * 12.0 + (double)ma.nnz21 * (4.0 + 4.0 * D) + (double)ma.nnzv * 4.0 * D +
                     (double)ma.n2 * 24.0;
  const double ndof = (double)D * ma.n2 + ma.nv;
  ProfScope ps(prof, s, "k_full_apply32", mat + b.nact * ndof * (8.0 + 16.0));
  k_full<D, SPMV_APPLY, false, float><<<nb, 256, 0, s>>>(ma, b, lm, x, y, VArg{}, nullptr, 0, nullptr);
  launch_check(s);
}

// y = A x for the interleaved preconditioner output (FP64 or FP32 values by R).
template <int D, class R, class YT>
void full_launch_il(Profiler* prof, const MeshArgs& ma, const S2SellArgs* sa, const Batch& b,
                    const typename Prec<R>::C* xil, SV<YT> y, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nb = row_blocks(ma.n2, lm);
  const double vb = sizeof(R);  // bytes per real matrix value
  const double mat = (double)ma.nnz * (4.0 + 2.0 * vb) + (double)ma.nnz21 * (4.0 + vb * D) +
                     (double)ma.nnzv * vb * D + (double)ma.n2 * 24.0;
  const double ndof = (double)D * ma.n2 + ma.nv;
  ProfScope ps(prof, s, sizeof(R) == 4 ? "k_full_apply32" : "k_full_apply",
               mat + b.nact * ndof * (2.0 * vb + (double)sizeof(YT)));
  if constexpr (sizeof(R) == 4) {
    if (sa && (b.nact * D) % 2 == 0 && b.nact * D > 4 && b.nact * D <= 8) {  // four lanes, two pairs each
      const unsigned nbs = (unsigned)((sa->nslot + 63) / 64);
      k_full_sell4<D, YT><<<nbs, 256, 0, s>>>(ma, *sa, b, xil, y);
      launch_check(s);
      return;
    }
    if (sa) {  // sliced rows: W lanes per row (a power of two >= the systems, <= 64)
      int W = 1;
      while (W < b.nact && W < 64) W <<= 1;
      const int RW = 64 / W;
      const unsigned nbs = (unsigned)((sa->nslot + 4 * RW - 1) / (4 * RW));
      k_full_sell<D, YT><<<nbs, 256, 0, s>>>(ma, *sa, b, W, RW, xil, y);
      launch_check(s);
      return;
    }
  }
  k_full<D, SPMV_APPLY, false, R, true, YT><<<nb, 256, 0, s>>>(ma, b, lm, typename Prec<R>::V{}, y, VArg{}, nullptr,
                                                               0, nullptr, xil);
  launch_check(s);
}

template <int D, class VI>
void precond_launch(scvs_mesh m, Profiler* prof, const MeshArgs& ma, const Batch& b, const PrecondArgs& pa, SV<VI> v,
                    VArg z, void* zil, hipStream_t s) {
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nbu = row_blocks(ma.n2, lm);
  const unsigned nbp = (unsigned)((ma.nv * b.nact + 255) / 256);  // k_pstep: one thread per (vertex, system)
  const double n2 = (double)ma.n2, nv = (double)ma.nv, DN = (double)D * ma.n2, na = b.nact;
  dim3 gp((unsigned)((ma.nv + 255) / 256), (unsigned)b.nact);
  // interleaved pressure temporaries inside the slot pool's block (4 * nv per slot, contiguous)
  // (FP32 recurrence in mixed mode: the same temporaries hold float2 values)
  const ITemps<double2> ptl{pa.pt.p, ma.nv, b.nact};
  const ITemps<float2> ptl32{reinterpret_cast<float2*>(pa.pt.p), ma.nv, b.nact};
  const double pes = pa.mixed ? 8.0 : 16.0, pvs = pa.mixed ? 4.0 : 8.0;  // complex / real temp bytes
  {
    // per system: v_p read, r/d0/x written (and z_p when one step); lpdinv, Mp read
    ProfScope ps(prof, s, pa.mixed ? "k_pinit32" : "k_pinit", nv * 16.0 + na * nv * (16.0 + 2.0 * pes));
    // (multigrid: the first smoothing iterate of the Laplacian's level 0, smoother interval)
    const double rp = pa.pmg ? pa.mg_ratio : pa.ratio_p;
    const int kp = pa.pmg ? 2 : pa.kp;
    if (pa.mixed)
      k_pinit<VI, float><<<gp, 256, 0, s>>>(ma, D, b, v, z, ptl32, rp, kp);
    else
      k_pinit<VI, double><<<gp, 256, 0, s>>>(ma, D, b, v, z, ptl, rp, kp);
  }
  if (pa.pmg) mg_pressure(m, b, pa, v, z, s);
  // L values and columns, row pointers, diag, Mp; per system x_i gathered (read once),
  // b and x_{i-1} read, x_{i+1} written (last step: v_p read and z_p written instead)
  const double pbytes = (double)ma.nnzl * (4.0 + pvs) + nv * 24.0 + na * nv * pes * 4.0;
  if (!pa.pmg && pa.kp > 1) {
    // the steps run back to back: one timed span for all of them
    ProfScope ps(prof, s, pa.mixed ? "k_pstep32" : "k_pstep", pbytes * (pa.kp - 1) + na * nv * (32.0 - pes),
                 pa.kp - 1);
    for (int i = 1; i < pa.kp; ++i) {
      if (pa.mixed)
        k_pstep<VI, float><<<nbp, 256, 0, s>>>(ma, D, b, v, z, ptl32, pa.ratio_p, cheb_step(pa.ratio_p, i), i,
                                               i == pa.kp - 1);
      else
        k_pstep<VI, double><<<nbp, 256, 0, s>>>(ma, D, b, v, z, ptl, pa.ratio_p, cheb_step(pa.ratio_p, i), i,
                                                i == pa.kp - 1);
    }
  }
  const double es = pa.mixed ? 8.0 : 16.0, vs = pa.mixed ? 4.0 : 8.0;  // complex / real element bytes
  // interleaved temporaries inside the slot pool's temp block (4 * D*n2 per slot, contiguous)
  const ITemps<double2> it64{pa.vt.p, ma.n2, lm.G};
  const ITemps<float2> it32{pa.vt32.p, ma.n2, lm.G};
  {
    // vertex-column prefix (col + G), row arrays; per system v_u read (FP64), z_p read (FP64),
    // b and x_1 written (and the FP32 copy of z_p in mixed mode)
    ProfScope ps(prof, s, pa.mixed ? "k_vinit32" : "k_vinit",
                 (double)ma.nnz21 * (4.0 + vs * D) + n2 * (24.0 + 2.0 * vs) +
                     na * (DN * 16.0 + nv * 16.0 + 2.0 * DN * es + (pa.mixed ? nv * es : 0.0)));
    if (pa.vmg) {
      // multigrid: b and the first smoothing iterate of level 0 (complex diagonal)
      Batch bv = b;
      bv.lv = pa.mg.vlam;
      const Sell& S = m->s2sell;
      if (pa.mixed && zil && S.K32.p && m->s2_G32.p) {
        int W = 1;
        while (W < b.nact && W < 64) W <<= 1;
        const int RW = 64 / W;
        const S2SellArgs sa{S.nslot, S.split_slots, S.off, m->s2_goff, S.row, S.col, S.K32, S.M32, m->s2_G32,
                            m->s2_Gt32};
        k_vinit_sell<D, VI><<<(unsigned)((S.nslot + 4 * RW - 1) / (4 * RW)), 256, 0, s>>>(
            ma, sa, bv, W, RW, v, z, it32, pa.mg_ratio, (float2*)zil);
      } else if (pa.mixed)
        k_vinit<D, float, VI, true><<<nbu, 256, 0, s>>>(ma, bv, lm, v, z, pa.z32, it32, pa.mg_ratio, 2, (float2*)zil);
      else
        k_vinit<D, double, VI, true><<<nbu, 256, 0, s>>>(ma, bv, lm, v, z, z, it64, pa.mg_ratio, 2, (double2*)zil);
    } else if (pa.mixed) {
      k_vinit<D, float, VI><<<nbu, 256, 0, s>>>(ma, b, lm, v, z, pa.z32, it32, pa.ratio, pa.kv, (float2*)zil);
    } else {
      k_vinit<D, double, VI><<<nbu, 256, 0, s>>>(ma, b, lm, v, z, z, it64, pa.ratio, pa.kv, (double2*)zil);
    }
  }
  if (pa.vmg) {
    launch_check(s);
    mg_velocity(m, b, pa, zil, z, s);
    return;
  }
  // S2 col/Ks/M, rowptr/dmask/Kd/Md; per system x_k (gathered, read once), b, x_{k-1} read, x_{k+1} written
  const double vbytes = (double)ma.nnz * (4.0 + 2.0 * vs) + n2 * (12.0 + 2.0 * vs) + na * 4.0 * DN * es;
  if (pa.kv > 1) {
    ProfScope ps(prof, s, pa.mixed ? "k_vstep32" : "k_vstep", vbytes * (pa.kv - 1), pa.kv - 1);
    for (int i = 1; i < pa.kv; ++i) {
      if (pa.mixed)
        k_vstep<D, float><<<nbu, 256, 0, s>>>(ma, b, lm, pa.z32, it32, pa.ratio, cheb_step(pa.ratio, i), i,
                                              i == pa.kv - 1, (float2*)zil);
      else
        k_vstep<D, double><<<nbu, 256, 0, s>>>(ma, b, lm, z, it64, pa.ratio, cheb_step(pa.ratio, i), i,
                                               i == pa.kv - 1, (double2*)zil);
    }
  }
  launch_check(s);
}

// y_slot = (float) x_slot for the active systems
__global__ void k_round32(const int* __restrict__ act, VArg x, VArg32 y, int64_t n) {
  const int slot = act[blockIdx.y];
  const double2* xs = x.at(slot);
  float2* ys = y.at(slot);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    ys[i] = make_float2((float)xs[i].x, (float)xs[i].y);
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

}  // namespace

void spmv_full(scvs_mesh m, const Batch& b, VArg x, VArg y, int mode, bool maskcol, VArg f, const double2* trac,
               hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  const int ntr = (int)m->traction_tags.size();
  if (m->dim == 2)
    full_launch<2>(&m->ctx->prof, ma, b, x, y, mode, maskcol, f, m->loads, ntr, trac, s);
  else
    full_launch<3>(&m->ctx->prof, ma, b, x, y, mode, maskcol, f, m->loads, ntr, trac, s);
  wk_launch<double2, false, double2>(m, b, mode, x, nullptr, y, s);
}

template <class VI>
static void precond_any(scvs_mesh m, const Batch& b, const PrecondArgs& pa, SV<VI> v, VArg z, hipStream_t s,
                        void* zil) {
  const MeshArgs ma = mesh_args(m);
  if (m->dim == 2)
    precond_launch<2, VI>(m, &m->ctx->prof, ma, b, pa, v, z, zil, s);
  else
    precond_launch<3, VI>(m, &m->ctx->prof, ma, b, pa, v, z, zil, s);
}

void precond_apply(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s, void* zil) {
  precond_any(m, b, pa, v, z, s, zil);
}

void precond_apply(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg32 v, VArg z, hipStream_t s, void* zil) {
  precond_any(m, b, pa, v, z, s, zil);
}

template <class YT>
static void spmv_il_any(scvs_mesh m, const Batch& b, const void* xil, bool fp32, SV<YT> y, hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  const Sell& S = m->s2sell;
  S2SellArgs sa{S.nslot, S.split_slots, S.off, m->s2_goff, S.row, S.col, S.K32, S.M32, m->s2_G32, m->s2_Gt32};
  const S2SellArgs* sp = (fp32 && S.K32.p && m->s2_G32.p) ? &sa : nullptr;
  if (m->dim == 2) {
    if (fp32)
      full_launch_il<2, float, YT>(&m->ctx->prof, ma, sp, b, (const float2*)xil, y, s);
    else
      full_launch_il<2, double, YT>(&m->ctx->prof, ma, nullptr, b, (const double2*)xil, y, s);
  } else {
    if (fp32)
      full_launch_il<3, float, YT>(&m->ctx->prof, ma, sp, b, (const float2*)xil, y, s);
    else
      full_launch_il<3, double, YT>(&m->ctx->prof, ma, nullptr, b, (const double2*)xil, y, s);
  }
  if (fp32)
    wk_launch<float2, true, YT>(m, b, SPMV_APPLY, SV<float2>{}, (const float2*)xil, y, s);
  else
    wk_launch<double2, true, YT>(m, b, SPMV_APPLY, SV<double2>{}, (const double2*)xil, y, s);
}

void spmv_apply_il(scvs_mesh m, const Batch& b, const void* xil, bool fp32, VArg y, hipStream_t s) {
  spmv_il_any(m, b, xil, fp32, y, s);
}

void spmv_apply_il(scvs_mesh m, const Batch& b, const void* xil, bool fp32, VArg32 y, hipStream_t s) {
  spmv_il_any(m, b, xil, fp32, y, s);
}

void spmv_resid32(scvs_mesh m, const Batch& b, VArg x, VArg32 y, VArg f, hipStream_t s, VArg tmp) {
  if (m->nwk > 0 && !b.no_lumped && tmp.p) {
    // with lumped outlets the operator part and the rank-one part nearly cancel near
    // convergence: form the residual in FP64 and round it once
    spmv_full(m, b, x, tmp, SPMV_RESID, true, f, nullptr, s);
    const int64_t ndof = (int64_t)m->dim * m->n2 + m->nv;
    k_round32<<<dim3(256, (unsigned)b.nact), 256, 0, s>>>(b.act, tmp, y, ndof);
    launch_check(s);
    return;
  }
  const MeshArgs ma = mesh_args(m);
  const int D = m->dim;
  const LaneMap lm = lane_map(b.nact, D);
  const unsigned nb = row_blocks(ma.n2, lm);
  const double ndof = (double)D * ma.n2 + ma.nv;
  ProfScope ps(&m->ctx->prof, s, "k_full_resid", full_bytes(ma, D, b.nact, SPMV_RESID) - b.nact * ndof * 8.0);
  if (D == 2)
    k_full<2, SPMV_RESID, true, double, false, float2><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, nullptr, 0, nullptr);
  else
    k_full<3, SPMV_RESID, true, double, false, float2><<<nb, 256, 0, s>>>(ma, b, lm, x, y, f, nullptr, 0, nullptr);
  launch_check(s);
  wk_launch<double2, false, float2>(m, b, SPMV_RESID, x, nullptr, y, s);
}

void spmv_apply32(scvs_mesh m, const Batch& b, VArg32 x, VArg y, hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  if (m->dim == 2)
    full_launch32<2>(&m->ctx->prof, ma, b, x, y, s);
  else
    full_launch32<3>(&m->ctx->prof, ma, b, x, y, s);
  wk_launch<float2, false, double2>(m, b, SPMV_APPLY, x, nullptr, y, s);
}

void make_fp32_copies(scvs_mesh m, hipStream_t s) {
  if (m->fp32_ready) return;
  const int D = m->dim;
  auto conv = [&](const DBuf<double>& a, DBuf<float>& b, size_t n) {
    b.alloc(n);
    k_to_f32<<<1024, 256, 0, s>>>(a.p, b.p, (int64_t)n);
    launch_check(s);
  };
  conv(m->Ks, m->Ks32, m->nnz);
  conv(m->M, m->M32, m->nnz);
  conv(m->G, m->G32, (size_t)D * m->nnz21);
  conv(m->Gt, m->Gt32, (size_t)D * m->nnzv);
  conv(m->Kd, m->Kd32, m->n2);
  conv(m->Md, m->Md32, m->n2);
  SCVS_HIP(hipStreamSynchronize(s));
  m->fp32_ready = true;
}

void velocity_bounds(scvs_mesh m, const Batch& b, double* lv_out, hipStream_t s) {
  const MeshArgs ma = mesh_args(m);
  dim3 g(256, (unsigned)b.nact);
  k_vbound<<<g, 256, 0, s>>>(ma, b, reinterpret_cast<unsigned long long*>(lv_out));
  launch_check(s);
}

}  // namespace scvs

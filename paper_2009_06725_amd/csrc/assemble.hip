// Element assembly of the mode-independent matrices (section 2.3, Eq. LS_construction):
//   Ks_AB = int grad M_A . grad M_B,   M_AB = int M_A M_B,   G^c_Av = -int d_c M_A N_v.
//
// Per cell and quadrature point the quadratic geometry map gives J, |det J| and
// J^-1. With C = J^-1 J^-T, W = w_q |det J| and reference gradients dM_A/dxi_k:
//   Ks_e[A][B] = sum_q sum_{k<=l} W C_kl (dM_A/dxi_k dM_B/dxi_l + [k!=l] dM_A/dxi_l dM_B/dxi_k)
//   M_e[A][B]  = sum_q W M_A M_B
//   G_e[c][A][v] = -sum_q sum_k W J^-1_kc dM_A/dxi_k N_v
// i.e. for a tile of 16 cells a dense product [16 x K] . [K x N] whose left
// factor is per-cell geometry and whose right factor is built from the LDS
// basis table. Those products run on the FP64 matrix cores (16x16x4). Element
// matrices are then summed into the CSR slots in ascending cell order.
#include <cmath>
#include <functional>

#include "internal.hpp"

namespace scvs {

void gm_rule(int n, int s, std::vector<double>& bary, std::vector<double>& w) {
  // Grundmann & Moeller (1978): degree d = 2s+1 on the n-simplex of volume 1/n!.
  const int d = 2 * s + 1;
  bary.clear();
  w.clear();
  auto fact = [](int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  };
  for (int i = 0; i <= s; ++i) {
    const int den = d + n - 2 * i;
    const double wi = ((i % 2) ? -1.0 : 1.0) * std::ldexp(1.0, -2 * s) * std::pow((double)den, d) /
                      (fact(i) * fact(d + n - i));
    std::vector<int> beta(n + 1, 0);
    std::function<void(int, int)> rec = [&](int pos, int left) {
      if (pos == n) {
        beta[n] = left;
        for (int k = 0; k <= n; ++k) bary.push_back((2.0 * beta[k] + 1.0) / den);
        w.push_back(wi);
        return;
      }
      for (int b = left; b >= 0; --b) {
        beta[pos] = b;
        rec(pos + 1, left - b);
      }
    };
    rec(0, s - i);
  }
}

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int D>
struct EL {
  static constexpr int NVL = D + 1;
  static constexpr int NN = (D + 1) * (D + 2) / 2;
  static constexpr int NQ = (D == 2) ? 10 : 15;  // Grundmann-Moeller degree 5
  static constexpr int NK = D * (D + 1) / 2;     // symmetric entries of C
  static constexpr int NF = NK + 1 + D * D;      // factors per quadrature point
  static constexpr int TS = 1 + NVL + NN + NN * D;  // table stride per point: w, lam, phi, dphi
  static constexpr int ESZ = 2 * NN * NN + D * NN * NVL + NVL;
};

// Lane layout of v_mfma_f64_16x16x4f64 used throughout:
//  A[i][k]: lane i + 16k;  B[k][j]: lane j + 16k;  D[i][j]: lane j + 16(i%4), element i/4
// (checked on the device by scvs_probe_mfma).
__device__ __forceinline__ v4d mfma16x16x4(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int D>
__global__ void __launch_bounds__(128) k_elements(const int32_t* __restrict__ c2n, int64_t nc, int64_t nv,
                                                  const double* __restrict__ xyz, const double* __restrict__ exyz,
                                                  const double* __restrict__ table, double* __restrict__ E) {
  using T = EL<D>;
  constexpr int NN = T::NN, NQ = T::NQ, NK = T::NK, NF = T::NF, TS = T::TS, NVL = T::NVL;
  __shared__ double tab[NQ * TS];
  __shared__ double F[2][16 * NQ * NF];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < NQ * TS; i += blockDim.x) tab[i] = table[i];
  __syncthreads();
  const int64_t cell0 = ((int64_t)blockIdx.x * 2 + wv) * 16;
  double* Fw = F[wv];
  constexpr int KL[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  constexpr int KL2[3][2] = {{0, 0}, {1, 1}, {0, 1}};
  // geometry factors for 16 cells x NQ points
  for (int p = lane; p < 16 * NQ; p += 64) {
    const int i = p / NQ, q = p % NQ;
    const int64_t c = cell0 + i;
    double* f = Fw + (i * NQ + q) * NF;
    if (c >= nc) {
      for (int k = 0; k < NF; ++k) f[k] = 0.0;
      continue;
    }
    const double* tq = tab + q * TS;
    double J[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int k = 0; k < D; ++k) J[r][k] = 0.0;
    for (int a = 0; a < NN; ++a) {
      const int32_t nd = c2n[c * NN + a];
      const double* X = (nd < nv) ? xyz + (int64_t)nd * D : exyz + (int64_t)(nd - nv) * D;
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const double xr = X[r];
#pragma unroll
        for (int k = 0; k < D; ++k) J[r][k] += xr * tq[1 + NVL + NN + a * D + k];
      }
    }
    double Ji[D][D], det;
    if constexpr (D == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const double id = 1.0 / det;
      Ji[0][0] = J[1][1] * id;
      Ji[0][1] = -J[0][1] * id;
      Ji[1][0] = -J[1][0] * id;
      Ji[1][1] = J[0][0] * id;
    } else {
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      const double id = 1.0 / det;
      Ji[0][0] = c00 * id;
      Ji[1][0] = c01 * id;
      Ji[2][0] = c02 * id;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    }
    const double W = tq[0] * fabs(det);
#pragma unroll
    for (int kl = 0; kl < NK; ++kl) {
      const int k = (D == 3) ? KL[kl][0] : KL2[kl][0];
      const int l = (D == 3) ? KL[kl][1] : KL2[kl][1];
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) s += Ji[k][r] * Ji[l][r];
      f[kl] = W * s;
    }
    f[NK] = W;
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int cc = 0; cc < D; ++cc) f[NK + 1 + k * D + cc] = W * Ji[k][cc];
  }
  __syncthreads();
  const int li = lane & 15, lk = lane >> 4;
  // ---- stiffness: K = NQ*NK, N = NN*NN ----
  {
    constexpr int KT = NQ * NK, KS = (KT + 3) / 4, NCOL = NN * NN, NT = (NCOL + 15) / 16;
    for (int t = 0; t < NT; ++t) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      const int j = t * 16 + li;
      const int A = j / NN, B = j % NN;
      for (int ks = 0; ks < KS; ++ks) {
        const int kap = ks * 4 + lk;
        double a = 0.0, b = 0.0;
        if (kap < KT) {
          const int q = kap / NK, kl = kap % NK;
          a = Fw[(li * NQ + q) * NF + kl];
          if (j < NCOL) {
            const int k = (D == 3) ? KL[kl][0] : KL2[kl][0];
            const int l = (D == 3) ? KL[kl][1] : KL2[kl][1];
            const double* dp = tab + q * TS + 1 + NVL + NN;
            b = dp[A * D + k] * dp[B * D + l];
            if (k != l) b += dp[A * D + l] * dp[B * D + k];
          }
        }
        acc = mfma16x16x4(a, b, acc);
      }
      if (j < NCOL) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t c = cell0 + 4 * r + lk;
          if (c < nc) E[c * T::ESZ + j] = acc[r];
        }
      }
    }
  }
  // ---- mass: K = NQ, N = NN*NN ----
  {
    constexpr int KS = (NQ + 3) / 4, NCOL = NN * NN, NT = (NCOL + 15) / 16;
    for (int t = 0; t < NT; ++t) {
      v4d acc = {0.0, 0.0, 0.0, 0.0};
      const int j = t * 16 + li;
      const int A = j / NN, B = j % NN;
      for (int ks = 0; ks < KS; ++ks) {
        const int q = ks * 4 + lk;
        double a = 0.0, b = 0.0;
        if (q < NQ) {
          a = Fw[(li * NQ + q) * NF + NK];
          if (j < NCOL) {
            const double* ph = tab + q * TS + 1 + NVL;
            b = ph[A] * ph[B];
          }
        }
        acc = mfma16x16x4(a, b, acc);
      }
      if (j < NCOL) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t c = cell0 + 4 * r + lk;
          if (c < nc) E[c * T::ESZ + NN * NN + j] = acc[r];
        }
      }
    }
  }
  // ---- coupling, one product per component c: K = NQ*D, N = NN*NVL ----
  {
    constexpr int KT = NQ * D, KS = (KT + 3) / 4, NCOL = NN * NVL, NT = (NCOL + 15) / 16;
    for (int cc = 0; cc < D; ++cc) {
      for (int t = 0; t < NT; ++t) {
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        const int j = t * 16 + li;
        const int A = j / NVL, v = j % NVL;
        for (int ks = 0; ks < KS; ++ks) {
          const int kap = ks * 4 + lk;
          double a = 0.0, b = 0.0;
          if (kap < KT) {
            const int q = kap / D, k = kap % D;
            a = Fw[(li * NQ + q) * NF + NK + 1 + k * D + cc];
            if (j < NCOL) {
              const double* tq = tab + q * TS;
              b = -tq[1 + NVL + NN + A * D + k] * tq[1 + v];
            }
          }
          acc = mfma16x16x4(a, b, acc);
        }
        if (j < NCOL) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t c = cell0 + 4 * r + lk;
            if (c < nc) E[c * T::ESZ + 2 * NN * NN + cc * NCOL + j] = acc[r];
          }
        }
      }
    }
  }
  // ---- lumped pressure mass per cell vertex: int N_v ----
  for (int p = lane; p < 16 * NVL; p += 64) {
    const int i = p / NVL, v = p % NVL;
    const int64_t c = cell0 + i;
    if (c >= nc) continue;
    double s = 0.0;
    for (int q = 0; q < NQ; ++q) s += Fw[(i * NQ + q) * NF + NK] * tab[q * TS + 1 + v];
    E[c * T::ESZ + 2 * NN * NN + D * NN * NVL + v] = s;
  }
}

// One thread per S2 slot (A,B): sum the element entries of every cell that
// contains both nodes, in ascending cell order.
template <int D>
__global__ void k_gather(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col, int64_t n2,
                         int64_t nnz, const int32_t* __restrict__ nvcnt, const int64_t* __restrict__ rowptr21,
                         int64_t nnz21, int64_t nnzv, int64_t nv, const int32_t* __restrict__ edges,
                         const int64_t* __restrict__ vc_ptr, const int32_t* __restrict__ vc,
                         const int32_t* __restrict__ cells, const int32_t* __restrict__ c2n,
                         const double* __restrict__ E, double* __restrict__ Ks, double* __restrict__ M,
                         double* __restrict__ G, double* __restrict__ Gt, double* __restrict__ Kd,
                         double* __restrict__ Md) {
  using T = EL<D>;
  constexpr int NN = T::NN, NVL = T::NVL, NCG = NN * NVL;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nnz) return;
  int64_t lo = 0, hi = n2;  // row: last r with rowptr[r] <= j
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (rowptr[mid] <= j)
      lo = mid;
    else
      hi = mid;
  }
  const int64_t A = lo;
  const int32_t Bn = col[j];
  int32_t a, b;
  if (A < nv) {
    a = (int32_t)A;
    b = -1;
  } else {
    a = edges[2 * (A - nv)];
    b = edges[2 * (A - nv) + 1];
  }
  double ks = 0.0, mm = 0.0, g[D], gt[D];
#pragma unroll
  for (int k = 0; k < D; ++k) g[k] = gt[k] = 0.0;
  for (int64_t i = vc_ptr[a]; i < vc_ptr[a + 1]; ++i) {
    const int64_t c = vc[i];
    if (b >= 0) {
      bool in = false;
#pragma unroll
      for (int k = 0; k < NVL; ++k) in |= (cells[c * NVL + k] == b);
      if (!in) continue;
    }
    int la = -1, lb = -1;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const int32_t nd = c2n[c * NN + k];
      if (nd == (int32_t)A) la = k;
      if (nd == Bn) lb = k;
    }
    if (la < 0 || lb < 0) continue;
    const double* e = E + c * T::ESZ;
    ks += e[la * NN + lb];
    mm += e[NN * NN + la * NN + lb];
    if (lb < NVL) {
#pragma unroll
      for (int k = 0; k < D; ++k) g[k] += e[2 * NN * NN + k * NCG + la * NVL + lb];
    }
    if (la < NVL) {
#pragma unroll
      for (int k = 0; k < D; ++k) gt[k] += e[2 * NN * NN + k * NCG + lb * NVL + la];
    }
  }
  Ks[j] = ks;
  M[j] = mm;
  const int64_t jr = j - rowptr[A];
  if (jr < nvcnt[A]) {
#pragma unroll
    for (int k = 0; k < D; ++k) G[k * nnz21 + rowptr21[A] + jr] = g[k];
  }
  if (A < nv) {
#pragma unroll
    for (int k = 0; k < D; ++k) Gt[k * nnzv + j] = gt[k];
  }
  if (Bn == (int32_t)A) {
    Kd[A] = ks;
    Md[A] = mm;
  }
}

template <int D>
__global__ void k_mp(const int64_t* __restrict__ vc_ptr, const int32_t* __restrict__ vc,
                     const int32_t* __restrict__ cells, const double* __restrict__ E, int64_t nv,
                     double* __restrict__ Mp) {
  using T = EL<D>;
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  for (int64_t i = vc_ptr[v]; i < vc_ptr[v + 1]; ++i) {
    const int64_t c = vc[i];
    int lv = 0;
#pragma unroll
    for (int k = 0; k < T::NVL; ++k)
      if (cells[c * T::NVL + k] == (int32_t)v) lv = k;
    s += E[c * T::ESZ + 2 * T::NN * T::NN + D * T::NN * T::NVL + lv];
  }
  Mp[v] = s;
}

__global__ void k_probe(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ d) {
  const int lane = threadIdx.x;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  acc = mfma16x16x4(a[li * 4 + lk], b[lk * 16 + li], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) d[(4 * r + lk) * 16 + li] = acc[r];
}

template <int D>
std::vector<double> basis_table() {
  using T = EL<D>;
  std::vector<double> bary, w;
  gm_rule(D, 2, bary, w);
  const int nq = (int)w.size();
  if (nq != T::NQ) fail(SCVS_E_INVALID, "unexpected quadrature size");
  std::vector<double> tab(nq * T::TS, 0.0);
  const int le[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
  for (int q = 0; q < nq; ++q) {
    const double* l = &bary[q * (D + 1)];
    double* t = &tab[q * T::TS];
    t[0] = w[q];
    for (int v = 0; v <= D; ++v) t[1 + v] = l[v];
    double* ph = t + 1 + T::NVL;
    double* dp = ph + T::NN;
    double dl[10][4] = {};  // d phi / d lam
    for (int v = 0; v <= D; ++v) {
      ph[v] = l[v] * (2.0 * l[v] - 1.0);
      dl[v][v] = 4.0 * l[v] - 1.0;
    }
    for (int e = 0; e < T::NN - T::NVL; ++e) {
      const int i = le[e][0], j = le[e][1];
      ph[T::NVL + e] = 4.0 * l[i] * l[j];
      dl[T::NVL + e][i] = 4.0 * l[j];
      dl[T::NVL + e][j] = 4.0 * l[i];
    }
    for (int a = 0; a < T::NN; ++a)
      for (int k = 0; k < D; ++k) dp[a * D + k] = dl[a][k + 1] - dl[a][0];
  }
  return tab;
}

template <int D>
void assemble_impl(scvs_mesh m, hipStream_t s) {
  using T = EL<D>;
  std::vector<double> tab = basis_table<D>();
  DBuf<double> dtab, E;
  dtab.upload(tab.data(), tab.size(), s);
  E.alloc((size_t)m->nc * T::ESZ);
  const unsigned nb = (unsigned)((m->nc + 31) / 32);
  if (m->nc) {
    k_elements<D><<<nb, 128, 0, s>>>(m->c2n, m->nc, m->nv, m->xyz, m->exyz, dtab, E);
    SCVS_HIP(hipGetLastError());
  }
  m->Ks.alloc(m->nnz);
  m->M.alloc(m->nnz);
  m->G.alloc((size_t)D * m->nnz21);
  m->Gt.alloc((size_t)D * m->nnzv);
  m->Kd.alloc(m->n2);
  m->Md.alloc(m->n2);
  m->Mp.alloc(m->nv);
  k_gather<D><<<(unsigned)((m->nnz + 255) / 256), 256, 0, s>>>(
      m->rowptr, m->col, m->n2, m->nnz, m->nvc, m->rowptr21, m->nnz21, m->nnzv, m->nv, m->edges, m->vc_ptr, m->vc,
      m->cells, m->c2n, E, m->Ks, m->M, m->G, m->Gt, m->Kd, m->Md);
  SCVS_HIP(hipGetLastError());
  k_mp<D><<<(unsigned)((m->nv + 255) / 256), 256, 0, s>>>(m->vc_ptr, m->vc, m->cells, E, m->nv, m->Mp);
  SCVS_HIP(hipGetLastError());
  SCVS_HIP(hipStreamSynchronize(s));
}

}  // namespace

void assemble_mesh(scvs_mesh m, hipStream_t s) {
  if (m->dim == 2)
    assemble_impl<2>(m, s);
  else
    assemble_impl<3>(m, s);
}

void probe_mfma(const double* a, const double* b, double* d, hipStream_t s) {
  DBuf<double> da, db, dd;
  da.upload(a, 64, s);
  db.upload(b, 64, s);
  dd.alloc(256);
  k_probe<<<1, 64, 0, s>>>(da, db, dd);
  SCVS_HIP(hipGetLastError());
  download(d, dd.p, 256, s);
}

}  // namespace scvs

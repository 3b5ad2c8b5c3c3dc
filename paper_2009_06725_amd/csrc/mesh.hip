// Quadratic-node numbering, sparsity patterns and boundary data on the device.
//
// Numbering (section 2.3, Eq. shape_fun, with this library's reading): vertex
// nodes keep their index; edge nodes follow in lexicographic (a<b) order. All
// lists are built by per-row sort+unique in LDS, so the result does not depend
// on thread scheduling and matches a plain sort of the connectivity bit for bit.
#include <climits>

#include "internal.hpp"

namespace scvs {
namespace {

constexpr int ROW_BS = 64;     // one wavefront per row
constexpr int ROW_CAP = 4096;  // candidate entries per row held in LDS

// Sort sh[0..n) (padding to a power of two), then count the unique values
// (and those below `lim`); when `out` is set, write them in order.
__device__ int wave_sort_unique(int32_t* sh, int n, int32_t* out, int32_t lim, int* nlow,
                                int* scan) {
  const int t = threadIdx.x;
  int P = 1;
  while (P < n) P <<= 1;
  for (int i = n + t; i < P; i += ROW_BS) sh[i] = INT_MAX;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < P; i += ROW_BS) {
        int l = i ^ j;
        if (l > i) {
          int32_t a = sh[i], b = sh[l];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            sh[i] = b;
            sh[l] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  const int per = (n + ROW_BS - 1) / ROW_BS;
  const int b0 = t * per, b1 = min(n, b0 + per);
  int cnt = 0, low = 0;
  for (int i = b0; i < b1; ++i) {
    bool f = (i == 0) || (sh[i] != sh[i - 1]);
    cnt += f;
    low += (f && sh[i] < lim);
  }
  scan[t] = cnt;
  scan[ROW_BS + t] = low;
  __syncthreads();
  for (int off = 1; off < ROW_BS; off <<= 1) {
    int a = (t >= off) ? scan[t - off] : 0;
    int b = (t >= off) ? scan[ROW_BS + t - off] : 0;
    __syncthreads();
    scan[t] += a;
    scan[ROW_BS + t] += b;
    __syncthreads();
  }
  if (out) {
    int k = scan[t] - cnt;
    for (int i = b0; i < b1; ++i)
      if ((i == 0) || (sh[i] != sh[i - 1])) out[k++] = sh[i];
  }
  int total = scan[ROW_BS - 1];
  *nlow = scan[2 * ROW_BS - 1];
  __syncthreads();
  return total;
}

// Sorted neighbours b > a of every vertex a (these pairs are the edges).
__global__ void __launch_bounds__(ROW_BS) k_vn_rows(int nvl, const int32_t* __restrict__ cells,
                                                    const int64_t* __restrict__ vc_ptr,
                                                    const int32_t* __restrict__ vc, int64_t nv,
                                                    int32_t* __restrict__ cnt,
                                                    const int64_t* __restrict__ vn_ptr,
                                                    int32_t* __restrict__ vn, int* err) {
  __shared__ int32_t sh[ROW_CAP];
  __shared__ int scan[2 * ROW_BS];
  __shared__ int ncand;
  const int64_t a = blockIdx.x;
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  const int64_t cb = vc_ptr[a], L = vc_ptr[a + 1] - cb;
  for (int64_t i = threadIdx.x; i < L * nvl; i += ROW_BS) {
    int32_t v = cells[(int64_t)vc[cb + i / nvl] * nvl + (i % nvl)];
    if (v > a) {
      int pos = atomicAdd(&ncand, 1);
      if (pos < ROW_CAP) sh[pos] = v;
    }
  }
  __syncthreads();
  int n = ncand;
  if (n > ROW_CAP) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  int low;
  int u = wave_sort_unique(sh, n, vn ? vn + vn_ptr[a] : nullptr, INT_MAX, &low, scan);
  if (!vn && threadIdx.x == 0) cnt[a] = u;
}

// S2 row of quadratic node A: all nodes of the cells containing A.
__global__ void __launch_bounds__(ROW_BS) k_s2_rows(int nvl, int nn, const int32_t* __restrict__ cells,
                                                    const int32_t* __restrict__ c2n,
                                                    const int64_t* __restrict__ vc_ptr,
                                                    const int32_t* __restrict__ vc,
                                                    const int32_t* __restrict__ edges, int64_t nv,
                                                    int32_t* __restrict__ cnt, int32_t* __restrict__ nvc,
                                                    const int64_t* __restrict__ rowptr,
                                                    int32_t* __restrict__ col, int* err) {
  __shared__ int32_t sh[ROW_CAP];
  __shared__ int scan[2 * ROW_BS];
  __shared__ int ncand;
  const int64_t A = blockIdx.x;
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  int32_t a, b;
  if (A < nv) {
    a = (int32_t)A;
    b = -1;
  } else {
    a = edges[2 * (A - nv)];
    b = edges[2 * (A - nv) + 1];
  }
  const int64_t cb = vc_ptr[a], L = vc_ptr[a + 1] - cb;
  for (int64_t i = threadIdx.x; i < L * nn; i += ROW_BS) {
    const int64_t c = vc[cb + i / nn];
    bool inside = true;
    if (b >= 0) {
      inside = false;
      for (int k = 0; k < nvl; ++k) inside |= (cells[c * nvl + k] == b);
    }
    if (inside) {
      int pos = atomicAdd(&ncand, 1);
      if (pos < ROW_CAP) sh[pos] = c2n[c * nn + (i % nn)];
    }
  }
  __syncthreads();
  int n = ncand;
  if (n > ROW_CAP) {
    if (threadIdx.x == 0) atomicOr(err, 2);
    return;
  }
  int low;
  int u = wave_sort_unique(sh, n, col ? col + rowptr[A] : nullptr, (int32_t)nv, &low, scan);
  if (!col && threadIdx.x == 0) {
    cnt[A] = u;
    nvc[A] = low;
  }
}

__global__ void k_edges(const int64_t* __restrict__ vn_ptr, const int32_t* __restrict__ vn, int64_t nv,
                        int32_t* __restrict__ edges) {
  int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nv) return;
  for (int64_t e = vn_ptr[a]; e < vn_ptr[a + 1]; ++e) {
    edges[2 * e] = (int32_t)a;
    edges[2 * e + 1] = vn[e];
  }
}

// Edge id of the vertex pair (a, b) by binary search in a's neighbour row; -1 if absent.
__device__ __forceinline__ int64_t edge_id(const int64_t* __restrict__ vn_ptr, const int32_t* __restrict__ vn,
                                           int32_t a, int32_t b) {
  if (a > b) {
    int32_t t = a;
    a = b;
    b = t;
  }
  int64_t lo = vn_ptr[a], hi = vn_ptr[a + 1];
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (vn[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < vn_ptr[a + 1] && vn[lo] == b) ? lo : -1;
}

template <int D>
__global__ void k_c2n(const int32_t* __restrict__ cells, int64_t nc, const int64_t* __restrict__ vn_ptr,
                      const int32_t* __restrict__ vn, int64_t nv, int32_t* __restrict__ c2n) {
  constexpr int NVL = D + 1, NN = (D + 1) * (D + 2) / 2;
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int32_t v[NVL];
#pragma unroll
  for (int k = 0; k < NVL; ++k) v[k] = cells[c * NVL + k];
  const int le[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};
#pragma unroll
  for (int k = 0; k < NVL; ++k) c2n[c * NN + k] = v[k];
#pragma unroll
  for (int e = 0; e < NN - NVL; ++e)
    c2n[c * NN + NVL + e] = (int32_t)(nv + edge_id(vn_ptr, vn, v[le[e][0]], v[le[e][1]]));
}

template <int D>
__global__ void k_midpoints(const int32_t* __restrict__ edges, int64_t ne, const double* __restrict__ xyz,
                            double* __restrict__ exyz) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int32_t a = edges[2 * e], b = edges[2 * e + 1];
#pragma unroll
  for (int k = 0; k < D; ++k) exyz[e * D + k] = 0.5 * (xyz[a * D + k] + xyz[b * D + k]);
}

template <int D>
__global__ void k_fnodes(const int32_t* __restrict__ bfaces, int64_t nf, const int64_t* __restrict__ vn_ptr,
                         const int32_t* __restrict__ vn, int64_t nv, int32_t* __restrict__ fnodes, int* err) {
  constexpr int NFV = D, NFN = D * (D + 1) / 2;
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int32_t v[NFV];
#pragma unroll
  for (int k = 0; k < NFV; ++k) {
    v[k] = bfaces[f * NFV + k];
    fnodes[f * NFN + k] = v[k];
  }
  const int le[3][2] = {{0, 1}, {1, 2}, {0, 2}};
#pragma unroll
  for (int e = 0; e < NFN - NFV; ++e) {
    int64_t id = edge_id(vn_ptr, vn, v[le[e][0]], v[le[e][1]]);
    if (id < 0) atomicOr(err, 4);
    fnodes[f * NFN + NFV + e] = (int32_t)(nv + (id < 0 ? 0 : id));
  }
}

__global__ void k_set_midside(const int32_t* __restrict__ ev, const double* __restrict__ xyz, int64_t n, int dim,
                              const int64_t* __restrict__ vn_ptr, const int32_t* __restrict__ vn,
                              double* __restrict__ exyz, int* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t e = edge_id(vn_ptr, vn, ev[2 * i], ev[2 * i + 1]);
  if (e < 0) {
    atomicOr(err, 8);
    return;
  }
  for (int k = 0; k < dim; ++k) exyz[e * dim + k] = xyz[i * dim + k];
}

__global__ void k_mark(const int32_t* __restrict__ fnodes, const int32_t* __restrict__ fkind, int64_t nf,
                       int nfn, int kind, int32_t value, int32_t* __restrict__ dmask) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * nfn) return;
  if (fkind[i / nfn] == kind) dmask[fnodes[i]] = value;
}

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

__global__ void k_flag_eq(const int32_t* __restrict__ a, int64_t n, int32_t v, int32_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (a[i] == v);
}

__global__ void k_compact(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos, int64_t n,
                          int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (int32_t)i;
}

// Per facet: int psi_a n dGamma for its quadratic facet nodes (facet quadrature
// of degree 5 on the quadratic facet map). Out: fc[f][NFN][D].
template <int D>
__global__ void k_facet_loads(const int32_t* __restrict__ fnodes, int64_t nf, const double* __restrict__ xyz,
                              const double* __restrict__ exyz, int64_t nv, const double* __restrict__ qb,
                              const double* __restrict__ qw, int nq, double* __restrict__ fc) {
  constexpr int NFV = D, NFN = D * (D + 1) / 2;
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double X[NFN][D];
#pragma unroll
  for (int a = 0; a < NFN; ++a) {
    int32_t nd = fnodes[f * NFN + a];
#pragma unroll
    for (int k = 0; k < D; ++k) X[a][k] = (nd < nv) ? xyz[(int64_t)nd * D + k] : exyz[(int64_t)(nd - nv) * D + k];
  }
  double acc[NFN][D];
#pragma unroll
  for (int a = 0; a < NFN; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[a][k] = 0.0;
  const int le[3][2] = {{0, 1}, {1, 2}, {0, 2}};
  for (int q = 0; q < nq; ++q) {
    double mu[NFV];
#pragma unroll
    for (int k = 0; k < NFV; ++k) mu[k] = qb[q * NFV + k];
    double psi[NFN], dmu[NFN][NFV];  // d psi / d mu_k
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
      int i = le[e][0], j = le[e][1];
      psi[NFV + e] = 4.0 * mu[i] * mu[j];
      dmu[NFV + e][i] = 4.0 * mu[j];
      dmu[NFV + e][j] = 4.0 * mu[i];
    }
    double T[D - 1][D];
#pragma unroll
    for (int t = 0; t < D - 1; ++t)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NFN; ++a) s += X[a][k] * (dmu[a][t + 1] - dmu[a][0]);
        T[t][k] = s;
      }
    double nds[D];
    if constexpr (D == 2) {
      nds[0] = T[0][1];
      nds[1] = -T[0][0];
    } else {
      nds[0] = T[0][1] * T[1][2] - T[0][2] * T[1][1];
      nds[1] = T[0][2] * T[1][0] - T[0][0] * T[1][2];
      nds[2] = T[0][0] * T[1][1] - T[0][1] * T[1][0];
    }
    const double w = qw[q];
#pragma unroll
    for (int a = 0; a < NFN; ++a)
#pragma unroll
      for (int k = 0; k < D; ++k) acc[a][k] += w * psi[a] * nds[k];
  }
#pragma unroll
  for (int a = 0; a < NFN; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) fc[(f * NFN + a) * D + k] = acc[a][k];
}

// loads[A][k] = sum over facets f of tag `tag` containing A (ascending f) of fc.
template <int D>
__global__ void k_loads_gather(const int64_t* __restrict__ nf_ptr, const int32_t* __restrict__ nf_list,
                               const int32_t* __restrict__ fnodes, const int32_t* __restrict__ btags,
                               const double* __restrict__ fc, int64_t n2, int32_t tag,
                               double* __restrict__ loads) {
  constexpr int NFN = D * (D + 1) / 2;
  int64_t A = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= n2) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int64_t i = nf_ptr[A]; i < nf_ptr[A + 1]; ++i) {
    int64_t f = nf_list[i];
    if (btags[f] != tag) continue;
    int la = 0;
#pragma unroll
    for (int a = 0; a < NFN; ++a)
      if (fnodes[f * NFN + a] == A) la = a;
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += fc[(f * NFN + la) * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) loads[A * D + k] = acc[k];
}

// Pressure Laplacian of the Schur block, L = G_F^T diag(M)^-1 G_F with G_F the
// rows of G at free velocity nodes. Row v couples the vertices u of the C21 rows
// of the free nodes A in the S2 row of v (a distance-2 vertex pattern).
__global__ void __launch_bounds__(ROW_BS) k_lp_rows(const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ nvcnt,
                                                    const int32_t* __restrict__ dmask, int32_t* __restrict__ cnt,
                                                    const int64_t* __restrict__ lp_ptr,
                                                    int32_t* __restrict__ lp_col, int* err) {
  __shared__ int32_t sh[ROW_CAP];
  __shared__ int scan[2 * ROW_BS];
  __shared__ int ncand;
  const int64_t v = blockIdx.x;
  if (threadIdx.x == 0) ncand = 0;
  __syncthreads();
  for (int64_t j = rowptr[v] + threadIdx.x; j < rowptr[v + 1]; j += ROW_BS) {
    const int32_t A = col[j];
    if (dmask[A] != 0) continue;
    const int nA = nvcnt[A];
    const int pos = atomicAdd(&ncand, nA);
    for (int q = 0; q < nA; ++q)
      if (pos + q < ROW_CAP) sh[pos + q] = col[rowptr[A] + q];
  }
  __syncthreads();
  const int n = ncand;
  if (n > ROW_CAP) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  int low;
  const int u = wave_sort_unique(sh, n, lp_col ? lp_col + lp_ptr[v] : nullptr, INT_MAX, &low, scan);
  if (!lp_col && threadIdx.x == 0) cnt[v] = u;
}

// L[v][u] = sum over free A in the S2 row of v (ascending) of sum_c G^c_Av G^c_Au / M_AA.
template <int D>
__global__ void k_lp_vals(const int64_t* __restrict__ lp_ptr, const int32_t* __restrict__ lp_col, int64_t nnzl,
                          int64_t nv, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                          const int32_t* __restrict__ nvcnt, const int64_t* __restrict__ rowptr21,
                          const double* __restrict__ G, const double* __restrict__ Gt, int64_t nnz21, int64_t nnzv,
                          const double* __restrict__ Md, const int32_t* __restrict__ dmask,
                          double* __restrict__ lp_val) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnzl) return;
  int64_t lo = 0, hi = nv;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (lp_ptr[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  const int64_t v = lo;
  const int32_t u = lp_col[k];
  double sum = 0.0;
  for (int64_t j = rowptr[v]; j < rowptr[v + 1]; ++j) {
    const int32_t A = col[j];
    if (dmask[A] != 0) continue;
    int64_t a = rowptr[A], b = a + nvcnt[A];
    const int64_t base = a;
    while (a < b) {
      const int64_t mid = (a + b) >> 1;
      if (col[mid] < u)
        a = mid + 1;
      else
        b = mid;
    }
    if (a < base + nvcnt[A] && col[a] == u) {
      const int64_t q = a - base;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) s += Gt[c * nnzv + j] * G[c * nnz21 + rowptr21[A] + q];
      sum += s / Md[A];
    }
  }
  lp_val[k] = sum;
}

__global__ void k_lp_diag(const int64_t* __restrict__ lp_ptr, const int32_t* __restrict__ lp_col,
                          const double* __restrict__ lp_val, int64_t nv, double* __restrict__ lpdinv,
                          double* __restrict__ ratio) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double dg = 0.0, ra = 0.0;
  for (int64_t k = lp_ptr[v]; k < lp_ptr[v + 1]; ++k) {
    ra += fabs(lp_val[k]);
    if (lp_col[k] == (int32_t)v) dg = lp_val[k];
  }
  lpdinv[v] = dg > 0.0 ? 1.0 / dg : 0.0;
  ratio[v] = dg > 0.0 ? ra / dg : 0.0;
}

__global__ void k_max(const double* __restrict__ a, int64_t n, unsigned long long* out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, a[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

void check_err(const DBuf<int>& err, hipStream_t s, const char* what) {
  int e = 0;
  download(&e, err.p, 1, s);
  if (e & 3) fail(SCVS_E_CAPACITY, std::string(what) + ": a pattern row has more than 4096 candidate entries");
  if (e & 4) fail(SCVS_E_MESH, std::string(what) + ": a boundary facet edge is not an edge of any cell");
  if (e & 8) fail(SCVS_E_INVALID, std::string(what) + ": a curved midside pair is not an edge of the mesh");
}

}  // namespace

void mesh_build(scvs_mesh m, hipStream_t s) {
  const int D = m->dim;
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  // vertex -> cells
  build_adjacency(m->cells, m->nc, m->nvl, m->nv, m->vc_ptr, m->vc, s);
  // edges: sorted neighbours b > a
  DBuf<int32_t> cnt;
  cnt.alloc(m->nv);
  k_vn_rows<<<(unsigned)m->nv, ROW_BS, 0, s>>>(m->nvl, m->cells, m->vc_ptr, m->vc, m->nv, cnt, nullptr, nullptr, err);
  SCVS_HIP(hipGetLastError());
  check_err(err, s, "edge build");
  m->vn_ptr.alloc(m->nv + 1);
  m->ne = exclusive_scan32(cnt, m->vn_ptr, m->nv, s);
  m->vn.alloc(m->ne);
  k_vn_rows<<<(unsigned)m->nv, ROW_BS, 0, s>>>(m->nvl, m->cells, m->vc_ptr, m->vc, m->nv, nullptr, m->vn_ptr, m->vn, err);
  SCVS_HIP(hipGetLastError());
  m->n2 = m->nv + m->ne;
  m->edges.alloc(2 * m->ne);
  k_edges<<<nblk(m->nv), 256, 0, s>>>(m->vn_ptr, m->vn, m->nv, m->edges);
  m->c2n.alloc(m->nc * m->nn);
  m->exyz.alloc(m->ne * D);
  if (D == 2) {
    k_c2n<2><<<nblk(m->nc), 256, 0, s>>>(m->cells, m->nc, m->vn_ptr, m->vn, m->nv, m->c2n);
    k_midpoints<2><<<nblk(m->ne), 256, 0, s>>>(m->edges, m->ne, m->xyz, m->exyz);
  } else {
    k_c2n<3><<<nblk(m->nc), 256, 0, s>>>(m->cells, m->nc, m->vn_ptr, m->vn, m->nv, m->c2n);
    k_midpoints<3><<<nblk(m->ne), 256, 0, s>>>(m->edges, m->ne, m->xyz, m->exyz);
  }
  SCVS_HIP(hipGetLastError());
  // S2 rows (count pass, scan, fill pass)
  DBuf<int32_t> rcnt;
  rcnt.alloc(m->n2);
  m->nvc.alloc(m->n2);
  k_s2_rows<<<(unsigned)m->n2, ROW_BS, 0, s>>>(m->nvl, m->nn, m->cells, m->c2n, m->vc_ptr, m->vc, m->edges, m->nv,
                                               rcnt, m->nvc, nullptr, nullptr, err);
  SCVS_HIP(hipGetLastError());
  check_err(err, s, "pattern build");
  m->rowptr.alloc(m->n2 + 1);
  m->nnz = exclusive_scan32(rcnt, m->rowptr, m->n2, s);
  m->col.alloc(m->nnz);
  k_s2_rows<<<(unsigned)m->n2, ROW_BS, 0, s>>>(m->nvl, m->nn, m->cells, m->c2n, m->vc_ptr, m->vc, m->edges, m->nv,
                                               nullptr, nullptr, m->rowptr, m->col, err);
  SCVS_HIP(hipGetLastError());
  m->rowptr21.alloc(m->n2 + 1);
  m->nnz21 = exclusive_scan32(m->nvc, m->rowptr21, m->n2, s);
  download(&m->nnzv, m->rowptr.p + m->nv, 1, s);
  // boundary facets -> quadratic facet nodes, and node -> facets
  const int nfn = D * (D + 1) / 2;
  m->fnodes.alloc(m->nf * nfn);
  if (m->nf) {
    if (D == 2)
      k_fnodes<2><<<nblk(m->nf), 256, 0, s>>>(m->bfaces, m->nf, m->vn_ptr, m->vn, m->nv, m->fnodes, err);
    else
      k_fnodes<3><<<nblk(m->nf), 256, 0, s>>>(m->bfaces, m->nf, m->vn_ptr, m->vn, m->nv, m->fnodes, err);
    SCVS_HIP(hipGetLastError());
  }
  check_err(err, s, "facet build");
  build_adjacency(m->fnodes, m->nf, nfn, m->n2, m->nf_ptr, m->nf_list, s);
}

void mesh_set_midside(scvs_mesh m, int64_t n, const int32_t* ev, const double* xyz, hipStream_t s) {
  DBuf<int32_t> dev;
  DBuf<double> dx;
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  dev.upload(ev, 2 * n, s);
  dx.upload(xyz, n * m->dim, s);
  k_set_midside<<<nblk(n), 256, 0, s>>>(dev, dx, n, m->dim, m->vn_ptr, m->vn, m->exyz, err);
  SCVS_HIP(hipGetLastError());
  check_err(err, s, "set_midside");
}

void mesh_boundary(scvs_mesh m, hipStream_t s) {
  const int D = m->dim;
  const int nfn = D * (D + 1) / 2;
  std::vector<int32_t> tags_h(m->nf), fkind(m->nf, SCVS_BC_FREE);
  download(tags_h.data(), m->btags.p, m->nf, s);
  for (int64_t f = 0; f < m->nf; ++f)
    for (size_t k = 0; k < m->bc_tags.size(); ++k)
      if (m->bc_tags[k] == tags_h[f]) fkind[f] = m->bc_kinds[k];
  DBuf<int32_t> dk;
  dk.upload(fkind.data(), m->nf, s);
  m->dmask.alloc(m->n2);
  m->dmask.zero(s);
  if (m->nf) {
    k_mark<<<nblk(m->nf * nfn), 256, 0, s>>>(m->fnodes, dk, m->nf, nfn, SCVS_BC_DIRICHLET, 2, m->dmask);
    k_mark<<<nblk(m->nf * nfn), 256, 0, s>>>(m->fnodes, dk, m->nf, nfn, SCVS_BC_WALL, 1, m->dmask);
    SCVS_HIP(hipGetLastError());
  }
  DBuf<int32_t> flag;
  DBuf<int64_t> pos;
  flag.alloc(m->n2);
  pos.alloc(m->n2 + 1);
  k_flag_eq<<<nblk(m->n2), 256, 0, s>>>(m->dmask, m->n2, 2, flag);
  m->ndir = exclusive_scan32(flag, pos, m->n2, s);
  m->dirnodes.alloc(m->ndir);
  k_compact<<<nblk(m->n2), 256, 0, s>>>(flag, pos, m->n2, m->dirnodes);
  SCVS_HIP(hipGetLastError());
  // traction loads per traction tag (ascending tag order)
  m->traction_tags.clear();
  for (size_t k = 0; k < m->bc_tags.size(); ++k)
    if (m->bc_kinds[k] == SCVS_BC_TRACTION) m->traction_tags.push_back(m->bc_tags[k]);
  std::sort(m->traction_tags.begin(), m->traction_tags.end());
  const int ntr = (int)m->traction_tags.size();
  m->loads.alloc((size_t)std::max(1, ntr) * m->n2 * D);
  m->loads.zero(s);
  if (ntr && m->nf) {
    std::vector<double> qb, qw;
    gm_rule(D - 1, 2, qb, qw);
    const int nq = (int)qw.size();
    DBuf<double> dqb, dqw, fc;
    dqb.upload(qb.data(), qb.size(), s);
    dqw.upload(qw.data(), qw.size(), s);
    fc.alloc(m->nf * nfn * D);
    if (D == 2)
      k_facet_loads<2><<<nblk(m->nf), 256, 0, s>>>(m->fnodes, m->nf, m->xyz, m->exyz, m->nv, dqb, dqw, nq, fc);
    else
      k_facet_loads<3><<<nblk(m->nf), 256, 0, s>>>(m->fnodes, m->nf, m->xyz, m->exyz, m->nv, dqb, dqw, nq, fc);
    SCVS_HIP(hipGetLastError());
    for (int t = 0; t < ntr; ++t) {
      double* out = m->loads.p + (size_t)t * m->n2 * D;
      if (D == 2)
        k_loads_gather<2><<<nblk(m->n2), 256, 0, s>>>(m->nf_ptr, m->nf_list, m->fnodes, m->btags, fc, m->n2,
                                                      m->traction_tags[t], out);
      else
        k_loads_gather<3><<<nblk(m->n2), 256, 0, s>>>(m->nf_ptr, m->nf_list, m->fnodes, m->btags, fc, m->n2,
                                                      m->traction_tags[t], out);
      SCVS_HIP(hipGetLastError());
    }
    SCVS_HIP(hipStreamSynchronize(s));
  }
  m->bc_set = true;
}

void mesh_precond_setup(scvs_mesh m, hipStream_t s) {
  const int D = m->dim;
  DBuf<int> err;
  err.alloc(1);
  err.zero(s);
  DBuf<int32_t> cnt;
  cnt.alloc(m->nv);
  k_lp_rows<<<(unsigned)m->nv, ROW_BS, 0, s>>>(m->rowptr, m->col, m->nvc, m->dmask, cnt, nullptr, nullptr, err);
  SCVS_HIP(hipGetLastError());
  check_err(err, s, "pressure Laplacian pattern");
  m->lp_ptr.alloc(m->nv + 1);
  m->nnzl = exclusive_scan32(cnt, m->lp_ptr, m->nv, s);
  m->lp_col.alloc(m->nnzl);
  m->lp_val.alloc(m->nnzl);
  k_lp_rows<<<(unsigned)m->nv, ROW_BS, 0, s>>>(m->rowptr, m->col, m->nvc, m->dmask, nullptr, m->lp_ptr, m->lp_col,
                                               err);
  SCVS_HIP(hipGetLastError());
  if (D == 2)
    k_lp_vals<2><<<nblk(m->nnzl), 256, 0, s>>>(m->lp_ptr, m->lp_col, m->nnzl, m->nv, m->rowptr, m->col, m->nvc,
                                              m->rowptr21, m->G, m->Gt, m->nnz21, m->nnzv, m->Md, m->dmask,
                                              m->lp_val);
  else
    k_lp_vals<3><<<nblk(m->nnzl), 256, 0, s>>>(m->lp_ptr, m->lp_col, m->nnzl, m->nv, m->rowptr, m->col, m->nvc,
                                              m->rowptr21, m->G, m->Gt, m->nnz21, m->nnzv, m->Md, m->dmask,
                                              m->lp_val);
  SCVS_HIP(hipGetLastError());
  m->lp_val32.alloc(m->nnzl);
  k_d2f<<<nblk(m->nnzl), 256, 0, s>>>(m->lp_val, m->lp_val32, m->nnzl);
  SCVS_HIP(hipGetLastError());
  DBuf<double> ratio;
  ratio.alloc(m->nv);
  m->lpdinv.alloc(m->nv);
  k_lp_diag<<<nblk(m->nv), 256, 0, s>>>(m->lp_ptr, m->lp_col, m->lp_val, m->nv, m->lpdinv, ratio);
  SCVS_HIP(hipGetLastError());
  DBuf<unsigned long long> mx;
  mx.alloc(1);
  mx.zero(s);
  k_max<<<256, 256, 0, s>>>(ratio, m->nv, mx);
  SCVS_HIP(hipGetLastError());
  unsigned long long bits = 0;
  download(&bits, mx.p, 1, s);
  double v;
  memcpy(&v, &bits, sizeof(v));
  m->lp_lmax = v > 0.0 ? v : 1.0;
}

namespace {

// Entries of one load vector b [n2*D] on unknowns whose node has mask value `want`
// (0 free, 2 prescribed inflow): flag, then compact (dof, b) in unknown order.
__global__ void k_wk_flag(const double* __restrict__ b, const int32_t* __restrict__ dmask, int64_t n, int D,
                          int32_t want, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (b[i] != 0.0 && dmask[i / D] == want);
}

__global__ void k_wk_compact(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                             const double* __restrict__ b, int64_t n, int32_t* __restrict__ dof,
                             double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) {
    dof[pos[i]] = (int32_t)i;
    val[pos[i]] = b[i];
  }
}

}  // namespace

void mesh_windkessel(scvs_mesh m, int n, const int32_t* tags, const double* rp, const double* c, const double* rd,
                     hipStream_t s) {
  m->nwk = 0;
  m->wk_par.clear();
  m->wk_nrow = 0;
  if (n == 0) return;
  const int D = m->dim;
  const int64_t N = m->n2 * D;
  DBuf<int32_t> flag;
  DBuf<int64_t> pos;
  flag.alloc(N);
  pos.alloc(N + 1);
  std::vector<int64_t> qoff(1, 0);
  std::vector<int32_t> qdof;
  std::vector<double> qb;
  struct Ent {
    int32_t dof, out;
    double b;
  };
  std::vector<Ent> rows;
  for (int o = 0; o < n; ++o) {
    const int t = (int)(std::find(m->traction_tags.begin(), m->traction_tags.end(), tags[o]) -
                        m->traction_tags.begin());
    const double* bt = m->loads.p + (size_t)t * N;
    for (int want : {0, 2}) {  // free unknowns, then prescribed-inflow unknowns
      k_wk_flag<<<nblk(N), 256, 0, s>>>(bt, m->dmask, N, D, want, flag);
      SCVS_HIP(hipGetLastError());
      const int64_t cnt = exclusive_scan32(flag, pos, N, s);
      if (cnt) {
        DBuf<int32_t> dd;
        DBuf<double> dv;
        dd.alloc(cnt);
        dv.alloc(cnt);
        k_wk_compact<<<nblk(N), 256, 0, s>>>(flag, pos, bt, N, dd, dv);
        SCVS_HIP(hipGetLastError());
        const size_t at = qdof.size();
        qdof.resize(at + cnt);
        qb.resize(at + cnt);
        download(qdof.data() + at, dd.p, cnt, s);
        download(qb.data() + at, dv.p, cnt, s);
        if (want == 0)
          for (int64_t e = 0; e < cnt; ++e) rows.push_back({qdof[at + e], o, qb[at + e]});
      }
      qoff.push_back((int64_t)qdof.size());
    }
    m->wk_par.insert(m->wk_par.end(), {rp[o], c[o], rd[o]});
  }
  // rows: distinct free unknowns, each with its (outlet, b) pairs in outlet order
  std::stable_sort(rows.begin(), rows.end(), [](const Ent& a, const Ent& b) { return a.dof < b.dof; });
  std::vector<int64_t> roff(1, 0);
  std::vector<int32_t> rdof, rout;
  std::vector<double> rb;
  for (size_t e = 0; e < rows.size(); ++e) {
    if (e == 0 || rows[e].dof != rows[e - 1].dof) {
      if (e) roff.push_back((int64_t)e);
      rdof.push_back(rows[e].dof);
    }
    rout.push_back(rows[e].out);
    rb.push_back(rows[e].b);
  }
  roff.push_back((int64_t)rows.size());
  if (rows.empty()) roff.assign(1, 0);
  auto up = [&](auto& buf, const auto& v) {
    if (v.empty())
      buf.alloc(1);
    else
      buf.upload(v.data(), v.size(), s);
  };
  up(m->wk_dpar, m->wk_par);
  up(m->wk_qoff, qoff);
  up(m->wk_qdof, qdof);
  up(m->wk_qb, qb);
  up(m->wk_roff, roff);
  up(m->wk_rdof, rdof);
  up(m->wk_rout, rout);
  up(m->wk_rb, rb);
  SCVS_HIP(hipStreamSynchronize(s));
  m->wk_nrow = (int64_t)rdof.size();
  m->nwk = n;
}

}  // namespace scvs

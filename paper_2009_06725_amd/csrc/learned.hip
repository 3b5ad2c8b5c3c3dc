// Learned warm start: POD of the method's own mode solutions and a small MLP
// (frequency features -> POD coefficients) trained with the project's own kernels.
//
// POD: G = X^H X (FP64, tiled, deterministic two-stage reduction), Hermitian
// eigen-decomposition of the S x S matrix on the host (cyclic Jacobi), basis
// phi_i = X w_i / sqrt(lambda_i). The projection of snapshot s on phi_i is
// sqrt(lambda_i) conj(w_si), which gives the training targets directly.
// MLP: every matrix product runs on the BF16 matrix cores (16x16x16, operands
// rounded to bfloat16 from the FP32 values, FP32 accumulation); tanh hidden
// layers, linear output, mean-squared-error loss, Adam on FP32 master weights.
// Inference: c = MLP(features(w)) scaled by the largest singular value, and
// x0 = a * sum_i c_i phi_i for each system (a = inlet amplitude of the mode).
// Optional subspace correction: x0 += Phi d with d minimizing the residual
// ||f - A(w)(x0 + Phi d)|| over the unconstrained rows; A(w) Phi is affine in
// w, so A(0) Phi and the w-slope are formed once per assembly and every
// system costs one residual, one projection and an r x r solve.
#include <cmath>
#include <complex>
#include <random>

#include "internal.hpp"

namespace scvs {

// ---- host: Hermitian eigen-decomposition by cyclic Jacobi ----
// A (n x n, row-major, Hermitian) is overwritten; on return w holds the
// eigenvalues (descending) and V (row-major, columns = eigenvectors).
void herm_eig(int n, std::vector<std::complex<double>>& A, std::vector<double>& w,
              std::vector<std::complex<double>>& V) {
  using cd = std::complex<double>;
  V.assign((size_t)n * n, cd(0.0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> cd& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double m2 = std::norm(a(i, j));
        tot += m2;
        if (i != j) off += m2;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd b = a(p, q);
        const double ab = std::abs(b);
        if (ab == 0.0) continue;
        // U = diag(1, e^{-i phi}) * [[c, -s], [s, c]] makes the (p,q) block diagonal
        const cd ph = b / ab;
        const double app = a(p, p).real(), aqq = a(q, q).real();
        const double theta = 0.5 * std::atan2(2.0 * ab, app - aqq);
        const double c = std::cos(theta), s = std::sin(theta);
        const cd u_pp = c, u_pq = -s, u_qp = s * std::conj(ph), u_qq = c * std::conj(ph);
        // columns: A <- A U
        for (int k = 0; k < n; ++k) {
          const cd akp = a(k, p), akq = a(k, q);
          a(k, p) = akp * u_pp + akq * u_qp;
          a(k, q) = akp * u_pq + akq * u_qq;
          const cd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = vkp * u_pp + vkq * u_qp;
          V[(size_t)k * n + q] = vkp * u_pq + vkq * u_qq;
        }
        // rows: A <- U^H A
        for (int k = 0; k < n; ++k) {
          const cd apk = a(p, k), aqk = a(q, k);
          a(p, k) = std::conj(u_pp) * apk + std::conj(u_qp) * aqk;
          a(q, k) = std::conj(u_pq) * apk + std::conj(u_qq) * aqk;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int i, int j) { return a(i, i).real() > a(j, j).real(); });
  std::vector<cd> V2((size_t)n * n);
  w.resize(n);
  for (int k = 0; k < n; ++k) {
    w[k] = a(idx[k], idx[k]).real();
    for (int i = 0; i < n; ++i) V2[(size_t)i * n + k] = V[(size_t)i * n + idx[k]];
  }
  V.swap(V2);
}

namespace {

// ---- cross products P = A^H B, A = [Sa][N], B = [Sb][N] complex (row-major) ----
constexpr int GT = 64;   // rows per tile side
constexpr int GK = 16;   // elements per LDS stage
// grid: (tile pairs, chunks). Thread t owns the 4x4 sub-block (ti, tj) of a 64x64 tile;
// part[chunk][i][j] holds the chunk's partial sum (reduced in a fixed order later).
__global__ void __launch_bounds__(256) k_cross(const double2* __restrict__ A, int Sa, const double2* __restrict__ B,
                                               int Sb, int64_t N, int ntb, int64_t chunk,
                                               double2* __restrict__ part) {
  __shared__ double2 sa[GT][GK + 1];
  __shared__ double2 sb[GT][GK + 1];
  const int tp = blockIdx.x;
  const int ti0 = (tp / ntb) * GT, tj0 = (tp % ntb) * GT;
  const int64_t k0 = (int64_t)blockIdx.y * chunk, k1 = min(N, k0 + chunk);
  const int t = threadIdx.x, ri = (t / 16) * 4, rj = (t % 16) * 4;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int64_t kb = k0; kb < k1; kb += GK) {
    for (int e = t; e < GT * GK; e += 256) {
      const int r = e / GK, kk = e % GK;
      const int64_t k = kb + kk;
      const int ia = ti0 + r, ib = tj0 + r;
      sa[r][kk] = (ia < Sa && k < k1) ? A[(int64_t)ia * N + k] : make_double2(0.0, 0.0);
      sb[r][kk] = (ib < Sb && k < k1) ? B[(int64_t)ib * N + k] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GK; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sa[ri + a][kk];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sb[rj + b][kk];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[a][b].x += av[a].x * bv[b].x + av[a].y * bv[b].y;
          acc[a][b].y += av[a].x * bv[b].y - av[a].y * bv[b].x;
        }
    }
    __syncthreads();
  }
  double2* out = part + (int64_t)blockIdx.y * Sa * Sb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ti0 + ri + a, j = tj0 + rj + b;
      if (i < Sa && j < Sb) out[(int64_t)i * Sb + j] = acc[a][b];
    }
}

__global__ void k_cross_reduce(const double2* __restrict__ part, int nch, int64_t n, double2* __restrict__ P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double2 s = make_double2(0.0, 0.0);
  for (int c = 0; c < nch; ++c) s = cadd(s, part[(int64_t)c * n + e]);
  P[e] = s;
}

// Q1 <- -j (Q1 - Q0) (so that A(w) phi = Q0 + j w Q1), then both rows zeroed at constrained dofs
__global__ void k_reduced_split(double2* __restrict__ Q, int r, int64_t N, const int32_t* __restrict__ dmask,
                                int64_t DN, int D) {
  const int i = blockIdx.y;
  double2* q0 = Q + (int64_t)i * N;
  double2* q1 = Q + (int64_t)(r + i) * N;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    const bool con = n < DN && dmask[n / D] != 0;
    const double2 a = q0[n], b = q1[n];
    q0[n] = con ? make_double2(0.0, 0.0) : a;
    q1[n] = con ? make_double2(0.0, 0.0) : make_double2(b.y - a.y, -(b.x - a.x));
  }
}

// B_o[dof] = b for the free entries of lumped outlet o (B zeroed before)
__global__ void k_lumped_columns(const int64_t* __restrict__ qoff, const int32_t* __restrict__ qdof,
                                 const double* __restrict__ qb, double2* __restrict__ B, int64_t N) {
  const int o = blockIdx.y;
  double2* col = B + (int64_t)o * N;
  for (int64_t e = qoff[2 * o] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < qoff[2 * o + 1];
       e += (int64_t)gridDim.x * blockDim.x)
    col[qdof[e]] = make_double2(qb[e], 0.0);
}

// zero rows of constrained dofs in R [n][N]
__global__ void k_mask_rows(double2* __restrict__ R, int64_t N, const int32_t* __restrict__ dmask, int64_t DN,
                            int D) {
  double2* rs = R + (int64_t)blockIdx.y * N;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < DN; n += (int64_t)gridDim.x * blockDim.x)
    if (dmask[n / D] != 0) rs[n] = make_double2(0.0, 0.0);
}

// phi_i[n] = sum_s X_s[n] C[s][i]   (C = W diag(1/sigma)), i < r
__global__ void k_pod_basis(const double2* __restrict__ X, int64_t N, int S, const double2* __restrict__ C, int r,
                            double2* __restrict__ Phi) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int i0 = 0; i0 < r; i0 += 16) {
    double2 acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = make_double2(0.0, 0.0);
    for (int s = 0; s < S; ++s) {
      const double2 x = X[(int64_t)s * N + n];
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (i0 + k < r) acc[k] = cadd(acc[k], cmul(x, C[(int64_t)s * r + i0 + k]));
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (i0 + k < r) Phi[(int64_t)(i0 + k) * N + n] = acc[k];
  }
}

// x0_s[n] (+)= sum_i coef[s][i] phi_i[n]   (coef already includes the amplitude)
__global__ void k_ws_combine(const double2* __restrict__ Phi, int64_t N, int r, const double2* __restrict__ coef,
                             double2* __restrict__ x0, int accumulate) {
  const int s = blockIdx.y;
  const double2* cs = coef + (int64_t)s * r;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = accumulate ? x0[(int64_t)s * N + n] : make_double2(0.0, 0.0);
    for (int i = 0; i < r; ++i) acc = cadd(acc, cmul(cs[i], Phi[(int64_t)i * N + n]));
    x0[(int64_t)s * N + n] = acc;
  }
}

// ---- BF16 matrix-core GEMM: C[M x N] = A[M x K] B[K x N] (+ bias[N]) ----
// A(i,k) = A[i*a_i + k*a_k], B(k,j) = B[k*b_k + j*b_j]; operands are FP32 in
// memory, rounded to bfloat16 (nearest even) when loaded; FP32 accumulation.
// Lane layout of v_mfma_f32_16x16x16_bf16 used here (checked on the device by
// scvs_probe_mfma_bf16): A[i][k] lane i + 16(k/4), element k%4; B[k][j] lane
// j + 16(k/4), element k%4; D[i][j] lane j + 16(i/4), element i%4.
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (short)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__global__ void __launch_bounds__(64) k_gemm_bf16(const float* __restrict__ A, int64_t a_i, int64_t a_k,
                                                  const float* __restrict__ B, int64_t b_k, int64_t b_j,
                                                  const float* __restrict__ bias, float* __restrict__ C, int M,
                                                  int N, int K) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.y * 16, j0 = blockIdx.x * 16;
  const int li = lane & 15, lq = lane >> 4;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4s a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + 4 * lq + e;
      const int i = i0 + li, j = j0 + li;
      const float av = (i < M && k < K) ? A[(int64_t)i * a_i + (int64_t)k * a_k] : 0.f;
      const float bv = (j < N && k < K) ? B[(int64_t)k * b_k + (int64_t)j * b_j] : 0.f;
      a[e] = to_bf16(av);
      b[e] = to_bf16(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = i0 + 4 * lq + e, j = j0 + li;
    if (i < M && j < N) C[(int64_t)i * N + j] = acc[e] + (bias ? bias[j] : 0.f);
  }
}

__global__ void k_probe_bf16(const float* __restrict__ a, const float* __restrict__ b, float* __restrict__ d) {
  const int lane = threadIdx.x, li = lane & 15, lq = lane >> 4;
  v4s av, bv;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    av[e] = to_bf16(a[li * 16 + 4 * lq + e]);
    bv[e] = to_bf16(b[(4 * lq + e) * 16 + li]);
  }
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
#pragma unroll
  for (int e = 0; e < 4; ++e) d[(4 * lq + e) * 16 + li] = acc[e];
}

__global__ void k_tanh(const float* __restrict__ z, float* __restrict__ h, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = tanhf(z[i]);
}

// dz = dh * (1 - h^2)
__global__ void k_dtanh(const float* __restrict__ dh, const float* __restrict__ h, float* __restrict__ dz,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = dh[i] * (1.f - h[i] * h[i]);
}

// dy = 2 (y - t) / n_all; per-block partial sums of (y - t)^2 (summed on the host in order)
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int64_t n, float* __restrict__ dy,
                      double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)n;
    s += (double)d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// gb[j] = sum_i dz[i][j]
__global__ void k_colsum(const float* __restrict__ dz, int n, int m, float* __restrict__ gb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += dz[(int64_t)i * m + j];
  gb[j] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// features of w: w/wmax, sqrt(w/wmax), (w/wmax)^2
__global__ void k_features(const double* __restrict__ omega, int n, double wmax, float* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = omega[i] / wmax;
  x[i * 3 + 0] = (float)w;
  x[i * 3 + 1] = (float)sqrt(fabs(w));
  x[i * 3 + 2] = (float)(w * w);
}

// coef[s][i] = amp_s * sigma_0 * (t_i + j t_{r+i}) with t_o = tmean_o + tscale_o out[s][o]
// (ts: tmean [2r] then tscale [2r])
__global__ void k_ws_coef(const float* __restrict__ out, int n, int r, double sigma0,
                          const double* __restrict__ ts, const double2* __restrict__ amp,
                          double2* __restrict__ coef) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * r) return;
  const int s = e / r, i = e % r;
  const double re = ts[i] + ts[2 * r + i] * (double)out[(int64_t)s * 2 * r + i];
  const double im = ts[r + i] + ts[3 * r + i] * (double)out[(int64_t)s * 2 * r + r + i];
  coef[e] = cmul(amp[s], make_double2(sigma0 * re, sigma0 * im));
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// P = A^H B (host, row-major [Sa][Sb]) for device A [Sa][N], B [Sb][N]; fixed-order reduction.
static std::vector<std::complex<double>> cross(scvs_ctx ctx, const double2* A, int Sa, const double2* B, int Sb,
                                               int64_t N, const char* name) {
  hipStream_t s = ctx->stream;
  const int nta = (Sa + GT - 1) / GT, ntb = (Sb + GT - 1) / GT;
  const int64_t np = (int64_t)Sa * Sb;
  // chunks along N: enough blocks to fill the chip, partial sums capped at 16M entries
  const int nch = (int)std::max<int64_t>(1, std::min<int64_t>({256, N / 4096, (int64_t)(1 << 24) / np}));
  const int64_t chunk = (N + nch - 1) / nch;
  DBuf<double2> part, P;
  part.alloc((size_t)nch * np);
  P.alloc((size_t)np);
  {
    ProfScope ps(&ctx->prof, s, name, (double)N * 16.0 * (Sa * ntb + Sb * nta));
    k_cross<<<dim3((unsigned)(nta * ntb), (unsigned)nch), 256, 0, s>>>(A, Sa, B, Sb, N, ntb, chunk, part);
  }
  k_cross_reduce<<<nb256(np), 256, 0, s>>>(part, nch, np, P);
  launch_check(s);
  std::vector<std::complex<double>> h((size_t)np);
  download(reinterpret_cast<double2*>(h.data()), P.p, (size_t)np, s);
  return h;
}

static void gemm(const float* A, int64_t a_i, int64_t a_k, const float* B, int64_t b_k, int64_t b_j,
                 const float* bias, float* C, int M, int N, int K, hipStream_t s) {
  dim3 g((unsigned)((N + 15) / 16), (unsigned)((M + 15) / 16));
  k_gemm_bf16<<<g, 64, 0, s>>>(A, a_i, a_k, B, b_k, b_j, bias, C, M, N, K);
  launch_check(s);
}

static const float* mlp_forward(Mlp& net, MlpWork& w, const float* x, int n, hipStream_t s) {
  const int L = net.layers();
  SCVS_HIP(hipMemcpyAsync(w.H[0].p, x, sizeof(float) * n * net.sizes[0], hipMemcpyDeviceToDevice, s));
  for (int l = 0; l < L; ++l) {
    const int in = net.sizes[l], out = net.sizes[l + 1];
    // Z = H W^T + b : A = H [n x in], B(k=in, j=out) = W[j][k]
    gemm(w.H[l].p, in, 1, net.p.p + net.woff[l], 1, in, net.p.p + net.boff[l], w.Z[l].p, n, out, in, s);
    if (l < L - 1) {
      k_tanh<<<nb256((int64_t)n * out), 256, 0, s>>>(w.Z[l].p, w.H[l + 1].p, (int64_t)n * out);
    } else {
      SCVS_HIP(hipMemcpyAsync(w.H[l + 1].p, w.Z[l].p, sizeof(float) * n * out, hipMemcpyDeviceToDevice, s));
    }
  }
  launch_check(s);
  return w.H[L].p;
}

// Loss and gradients (into net.g) for inputs x [n][in], targets t [n][out] (device).
static double mlp_loss_grad(Mlp& net, MlpWork& w, const float* x, const float* t, int n, hipStream_t s) {
  const int L = net.layers();
  const float* y = mlp_forward(net, w, x, n, s);
  const int no = net.sizes[L];
  k_mse<<<256, 256, 0, s>>>(y, t, (int64_t)n * no, w.dH[L].p, w.part.p);
  for (int l = L - 1; l >= 0; --l) {
    const int in = net.sizes[l], out = net.sizes[l + 1];
    const float* dz = w.dH[l + 1].p;
    if (l < L - 1) {
      k_dtanh<<<nb256((int64_t)n * out), 256, 0, s>>>(w.dH[l + 1].p, w.H[l + 1].p, w.dZ.p, (int64_t)n * out);
      dz = w.dZ.p;
    }
    // gW [out x in] = dZ^T H : A(i=out, k=n) = dz[k*out + i], B(k=n, j=in) = H[k*in + j]
    gemm(dz, 1, out, w.H[l].p, in, 1, nullptr, net.g.p + net.woff[l], out, in, n, s);
    k_colsum<<<nb256(out), 256, 0, s>>>(dz, n, out, net.g.p + net.boff[l]);
    // dH_l [n x in] = dZ W : A = dz [n x out], B(k=out, j=in) = W[k][j]
    if (l > 0) gemm(dz, out, 1, net.p.p + net.woff[l], in, 1, nullptr, w.dH[l].p, n, in, out, s);
  }
  launch_check(s);
  std::vector<double> part(256);
  download(part.data(), w.part.p, 256, s);
  double loss = 0.0;
  for (double v : part) loss += v;
  return loss / ((double)n * no);
}

static void adam(Mlp& net, float lr, hipStream_t s) {
  net.step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)net.step), c2 = 1.f - std::pow(b2, (float)net.step);
  k_adam<<<nb256(net.nparam), 256, 0, s>>>(net.p, net.g, net.m, net.v, net.nparam, lr, b1, b2, 1e-8f, c1, c2);
  launch_check(s);
}

}  // namespace scvs

namespace scvs {

void ws_build(scvs_ws w, int64_t S, const double* omega, const double2* snaps, int r, int width, int layers,
              uint64_t seed) {
  hipStream_t s = w->mesh->ctx->stream;
  const int64_t N = w->ndof;
  w->S = (int)S;
  w->r = r;
  w->omega.assign(omega, omega + S);
  w->wmax = 0.0;
  for (double o : w->omega) w->wmax = std::max(w->wmax, std::fabs(o));
  if (w->wmax == 0.0) w->wmax = 1.0;
  // Gram matrix on the device
  std::vector<std::complex<double>> A = cross(w->mesh->ctx, snaps, (int)S, snaps, (int)S, N, "k_gram"), V;
  std::vector<double> lam;
  herm_eig((int)S, A, lam, V);
  // basis coefficients C[s][i] = W_si / sigma_i; snapshot s = sum_i sigma_i conj(W_si) phi_i, so its
  // coefficients relative to sigma_0 are t_si = sigma_i conj(W_si) / sigma_0 (real parts, then
  // imaginary parts). Each of the 2r outputs is standardized over the snapshots (mean removed,
  // divided by the RMS deviation; an output that does not vary keeps scale 1), so the network
  // fits every coefficient to the same relative accuracy. Without it the trailing coefficients,
  // small but on the basis vectors the operator amplifies most, carry the network's absolute error.
  w->sigma.resize(r);
  const double sig0 = S > 0 ? std::sqrt(std::max(lam[0], 0.0)) : 0.0;
  w->sigma0 = sig0;
  std::vector<std::complex<double>> C((size_t)S * r);
  std::vector<double> t((size_t)S * 2 * r, 0.0);
  for (int i = 0; i < r; ++i) {
    const double sg = i < S ? std::sqrt(std::max(lam[i], 0.0)) : 0.0;
    w->sigma[i] = sg;
    for (int64_t sn = 0; sn < S; ++sn) {
      const std::complex<double> wsi = i < S ? V[(size_t)sn * S + i] : 0.0;
      C[(size_t)sn * r + i] = sg > 0 ? wsi / sg : 0.0;
      const std::complex<double> ti = sig0 > 0 ? std::conj(wsi) * (sg / sig0) : 0.0;
      t[(size_t)sn * 2 * r + i] = ti.real();
      t[(size_t)sn * 2 * r + r + i] = ti.imag();
    }
  }
  w->tmean.assign(2 * r, 0.0);
  w->tscale.assign(2 * r, 1.0);
  w->targets.assign((size_t)S * 2 * r, 0.f);
  for (int o = 0; o < 2 * r; ++o) {
    double mu = 0.0, var = 0.0;
    for (int64_t sn = 0; sn < S; ++sn) mu += t[(size_t)sn * 2 * r + o];
    mu /= (double)std::max<int64_t>(S, 1);
    for (int64_t sn = 0; sn < S; ++sn) var += (t[(size_t)sn * 2 * r + o] - mu) * (t[(size_t)sn * 2 * r + o] - mu);
    const double sd = std::sqrt(var / (double)std::max<int64_t>(S, 1));
    w->tmean[o] = mu;
    w->tscale[o] = sd > 0.0 ? sd : 1.0;
    for (int64_t sn = 0; sn < S; ++sn)
      w->targets[(size_t)sn * 2 * r + o] = (float)((t[(size_t)sn * 2 * r + o] - mu) / w->tscale[o]);
  }
  std::vector<double> ts(w->tmean);  // host copy lives until the synchronize below
  ts.insert(ts.end(), w->tscale.begin(), w->tscale.end());
  w->tstd_d.upload(ts.data(), ts.size(), s);
  DBuf<double2> Cd;
  Cd.upload(reinterpret_cast<double2*>(C.data()), C.size(), s);
  w->basis.alloc((size_t)r * N);
  {
    ProfScope ps(&w->mesh->ctx->prof, s, "k_pod_basis", (double)N * 16.0 * (S * ((r + 15) / 16) + r));
    k_pod_basis<<<nb256(N), 256, 0, s>>>(snaps, N, (int)S, Cd, r, w->basis);
  }
  launch_check(s);
  w->sigma_d.upload(w->sigma.data(), r, s);
  // network and training data (features of the snapshot frequencies)
  std::vector<int> sizes = {3};
  for (int l = 0; l < layers - 1; ++l) sizes.push_back(width);
  sizes.push_back(2 * r);
  w->net.init(sizes, seed, s);
  DBuf<double> om;
  om.upload(omega, S, s);
  w->X.alloc((size_t)S * 3);
  k_features<<<nb256(S), 256, 0, s>>>(om, (int)S, w->wmax, w->X);
  w->T.upload(w->targets.data(), w->targets.size(), s);
  SCVS_HIP(hipStreamSynchronize(s));
}

double ws_train(scvs_ws w, int epochs, double lr) {
  hipStream_t s = w->mesh->ctx->stream;
  w->work.ensure(w->net, w->S);
  double loss = mlp_loss_grad(w->net, w->work, w->X, w->T, w->S, s);  // loss before the epoch
  for (int e = 0; e < epochs; ++e) {
    if (e > 0) loss = mlp_loss_grad(w->net, w->work, w->X, w->T, w->S, s);
    adam(w->net, (float)lr, s);
  }
  return loss;
}

void ws_predict(scvs_ws w, int64_t n, const double* omega, const double* amp, double2* x0) {
  hipStream_t s = w->mesh->ctx->stream;
  DBuf<double> om;
  DBuf<float> X;
  DBuf<double2> a, coef;
  om.upload(omega, n, s);
  a.upload(reinterpret_cast<const double2*>(amp), n, s);
  X.alloc((size_t)n * 3);
  k_features<<<nb256(n), 256, 0, s>>>(om, (int)n, w->wmax, X);
  w->work.ensure(w->net, (int)std::max<int64_t>(n, w->S));
  const float* y = mlp_forward(w->net, w->work, X, (int)n, s);
  coef.alloc((size_t)n * w->r);
  k_ws_coef<<<nb256(n * w->r), 256, 0, s>>>(y, (int)n, w->r, w->sigma0, w->tstd_d, a, coef);
  {
    ProfScope ps(&w->mesh->ctx->prof, s, "k_ws_combine", (double)w->ndof * 16.0 * (w->r + n));
    k_ws_combine<<<dim3(512, (unsigned)n), 256, 0, s>>>(w->basis, w->ndof, w->r, coef, x0, 0);
  }
  launch_check(s);
  SCVS_HIP(hipStreamSynchronize(s));
}

// Reduced operator of the current assembly: Q0 = A(0) Phi, Q1 = (A(1) - A(0)) Phi / j on
// unconstrained rows, both without the lumped-outlet terms (the rest of A is affine
// in w); B holds each lumped outlet's load vector on unconstrained rows, Cb = B^T Phi;
// H = [Q0; Q1; B]^H [Q0; Q1; B].
static void ws_reduced(scvs_ws w) {
  scvs_mesh m = w->mesh;
  if (w->red_gen == m->generation) return;
  hipStream_t s = m->ctx->stream;
  const int r = w->r;
  const int nb = m->nwk;
  const int64_t N = w->ndof;
  w->Q.alloc((size_t)(2 * r + nb) * N);
  std::vector<double> om(2 * r, 0.0);
  for (int i = r; i < 2 * r; ++i) om[i] = 1.0;
  std::vector<int> a(2 * r);
  for (int i = 0; i < 2 * r; ++i) a[i] = i % r;
  DBuf<double> omd;
  DBuf<int> act;
  omd.upload(om.data(), om.size(), s);
  act.upload(a.data(), a.size(), s);
  // slot k reads phi_{k mod r}: apply A(0) to the basis into Q0 and A(1) into Q1
  for (int half = 0; half < 2; ++half) {
    Batch b;
    b.nact = r;
    b.act = act.p + half * r;
    b.omega = omd.p + half * r;
    b.no_lumped = true;
    spmv_full(m, b, VArg{w->basis.p, N}, VArg{w->Q.p + (int64_t)half * r * N, N}, SPMV_APPLY, true,
              VArg{}, nullptr, s);
  }
  const int64_t DN = (int64_t)m->dim * m->n2;
  k_reduced_split<<<dim3(512, (unsigned)r), 256, 0, s>>>(w->Q, r, N, m->dmask, DN, m->dim);
  launch_check(s);
  w->Cb.clear();
  if (nb) {
    double2* B = w->Q.p + (int64_t)2 * r * N;
    SCVS_HIP(hipMemsetAsync(B, 0, (size_t)nb * N * sizeof(double2), s));
    k_lumped_columns<<<dim3(64, (unsigned)nb), 256, 0, s>>>(m->wk_qoff, m->wk_qdof, m->wk_qb, B, N);
    launch_check(s);
    w->Cb = cross(m->ctx, B, nb, w->basis, r, N, "k_ws_lumped");
  }
  w->nb = nb;
  w->H = cross(m->ctx, w->Q, 2 * r + nb, w->Q, 2 * r + nb, N, "k_gram");
  w->red_gen = m->generation;
}

void ws_refine(scvs_ws w, int64_t n, const double* omega, const double* traction, const void* g, double2* x0) {
  using cd = std::complex<double>;
  scvs_mesh m = w->mesh;
  hipStream_t s = m->ctx->stream;
  ws_reduced(w);
  const int r = w->r;
  const int64_t N = w->ndof, DN = (int64_t)m->dim * m->n2;
  // residual of the guess on unconstrained rows: R = f - A x0
  DBuf<double2> F, R;
  F.alloc((size_t)n * N);
  R.alloc((size_t)n * N);
  rhs_systems(m, n, omega, traction, g, F.p);
  {
    DBuf<double> omd;
    DBuf<int> act;
    std::vector<int> a(n);
    for (int64_t k = 0; k < n; ++k) a[k] = (int)k;
    omd.upload(omega, n, s);
    act.upload(a.data(), n, s);
    Batch b;
    b.nact = (int)n;
    b.act = act;
    b.omega = omd;
    spmv_full(m, b, VArg{x0, N}, VArg{R.p, N}, SPMV_RESID, true, VArg{F.p, N}, nullptr, s);
    k_mask_rows<<<dim3(512, (unsigned)n), 256, 0, s>>>(R, N, m->dmask, DN, m->dim);
    launch_check(s);
    SCVS_HIP(hipStreamSynchronize(s));
  }
  const int nw = 2 * r + w->nb;
  const std::vector<cd> B = cross(m->ctx, w->Q, nw, R, (int)n, N, "k_ws_project");  // [nw][n]
  // per system: min || R - [Q0; Q1; B] E d || with E = [I; j w I; diag(Z(w)) Cb], normal
  // equations E^H H E d = E^H B solved by eigen-decomposition
  std::vector<cd> coef((size_t)n * r);
  for (int64_t k = 0; k < n; ++k) {
    const double wk = omega[k];
    std::vector<cd> E((size_t)nw * r, cd(0.0));
    for (int i = 0; i < r; ++i) {
      E[(size_t)i * r + i] = 1.0;
      E[(size_t)(r + i) * r + i] = cd(0.0, wk);
    }
    for (int o = 0; o < w->nb; ++o) {
      const double rp = m->wk_par[3 * o], cc = m->wk_par[3 * o + 1], rd = m->wk_par[3 * o + 2];
      const cd Z = rp + rd / cd(1.0, wk * rd * cc);
      for (int i = 0; i < r; ++i) E[(size_t)(2 * r + o) * r + i] = Z * w->Cb[(size_t)o * r + i];
    }
    std::vector<cd> HE((size_t)nw * r, cd(0.0)), Mk((size_t)r * r, cd(0.0)), V;
    std::vector<cd> rhs(r, cd(0.0));
    for (int a = 0; a < nw; ++a)
      for (int c = 0; c < nw; ++c) {
        const cd h = w->H[(size_t)a * nw + c];
        for (int j = 0; j < r; ++j) HE[(size_t)a * r + j] += h * E[(size_t)c * r + j];
      }
    for (int i = 0; i < r; ++i) {
      for (int a = 0; a < nw; ++a) {
        const cd e = std::conj(E[(size_t)a * r + i]);
        if (e == cd(0.0)) continue;
        for (int j = 0; j < r; ++j) Mk[(size_t)i * r + j] += e * HE[(size_t)a * r + j];
        rhs[i] += e * B[(size_t)a * n + k];
      }
    }
    std::vector<double> lam;
    herm_eig(r, Mk, lam, V);
    const double cut = 1e-13 * std::max(lam[0], 0.0);
    for (int e = 0; e < r; ++e) {
      if (!(lam[e] > cut)) break;
      cd proj = 0.0;
      for (int i = 0; i < r; ++i) proj += std::conj(V[(size_t)i * r + e]) * rhs[i];
      proj /= lam[e];
      for (int i = 0; i < r; ++i) coef[(size_t)k * r + i] += V[(size_t)i * r + e] * proj;
    }
  }
  DBuf<double2> cd_;
  cd_.upload(reinterpret_cast<double2*>(coef.data()), coef.size(), s);
  {
    ProfScope ps(&m->ctx->prof, s, "k_ws_combine", (double)N * 16.0 * (r + 2 * n));
    k_ws_combine<<<dim3(512, (unsigned)n), 256, 0, s>>>(w->basis, N, r, cd_, x0, 1);
  }
  launch_check(s);
  SCVS_HIP(hipStreamSynchronize(s));
}

double ws_loss_grad(scvs_ws w, int n, const float* x_host, const float* t_host, float* grads_host) {
  hipStream_t s = w->mesh->ctx->stream;
  DBuf<float> X, T;
  X.upload(x_host, (size_t)n * w->net.sizes[0], s);
  T.upload(t_host, (size_t)n * w->net.sizes.back(), s);
  MlpWork wk;
  wk.ensure(w->net, n);
  const double loss = mlp_loss_grad(w->net, wk, X, T, n, s);
  download(grads_host, w->net.g.p, w->net.nparam, s);
  return loss;
}

void probe_mfma_bf16(const float* a, const float* b, float* d, hipStream_t s) {
  DBuf<float> da, db, dd;
  da.upload(a, 256, s);
  db.upload(b, 256, s);
  dd.alloc(256);
  k_probe_bf16<<<1, 64, 0, s>>>(da, db, dd);
  launch_check(s);
  download(d, dd.p, 256, s);
}

}  // namespace scvs

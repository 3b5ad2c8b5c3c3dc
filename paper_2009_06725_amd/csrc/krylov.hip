// Block-preconditioned restarted GMRES for a batch of mode systems on one mesh.
//
// The paper solves each mode's system with GMRES (Saad & Schultz 1986),
// adapted to complex arithmetic (section 2.3; section 3.1). Here, per system:
// right preconditioning, Arnoldi by classical Gram-Schmidt with a second pass
// only when the first one cancels more than 30% of the norm, complex Givens
// rotations, restart on the recomputed true residual f - A x, and stop when
// ||f - A x|| <= rtol ||f||.
//
// Storage is system-major: every system owns a slot with its basis V[m+1],
// its solution, right-hand side and temporaries, so that finished systems
// drop out of a batch without data movement. Dot products reduce within the
// 64-lane wavefront by shuffles, then across the workgroup in LDS, then over
// workgroups in a fixed order by the last workgroup to finish (no floating-
// point atomics: results are bit-reproducible).
#include <cmath>
#include <functional>
#include <map>

#include "internal.hpp"

namespace scvs {
namespace {

constexpr int MM = SCVS_MMAX;
constexpr int PSTRIDE = 2 * MM + 4;  // partial sums per (slot, chunk)
constexpr int RBS = 256;         // reduction block size
constexpr int JB = 8;            // basis vectors per accumulation group

struct SlotState {
  double2 H[(MM + 1) * MM];  // column j at H + (MM+1) j
  double2 sn[MM];
  double cs[MM];
  double2 gam[MM + 1];
  double2 y[MM];
  double2 h1[MM + 1], h2[MM + 1];
  double hs[MM + 1];  // scale of stored basis vector i (V_i is kept unnormalized)
  double2 Hu[(MM + 1) * MM];  // unrotated Hessenberg matrix (lagged orthogonalization)
  double2 gq;                 // lagged: <q_j, W>
  double sig, rho;            // lagged: norm of the reorthogonalized u_j; norm of the last first-pass vector
  double nrm0, fnorm, tolabs, beta;
  double tolcyc;              // a cycle also ends when its residual estimate falls below this
  int jstop, skip2, nonfinite, lastJ;
  unsigned int ticket[8];
};

struct KArgs {
  const int* act;
  SlotState* st;
  double2* part;
  int nch;
  int64_t ndof, ld;
  int m;
  double2* V;  // slot k, vector i at V + (k*(m+1) + i)*ld
  float2* V32;  // the same storage as FP32 pairs when the basis is kept in FP32
  double* info;  // per slot: rel, lastJ, nonfinite, beta
};

__device__ __forceinline__ double2* vec(const KArgs& a, int slot, int i) {
  return a.V + ((int64_t)slot * (a.m + 1) + i) * a.ld;
}

// Basis vector i of a slot in the storage precision VT (double2 or float2).
template <class VT>
__device__ __forceinline__ VT* vecT(const KArgs& a, int slot, int i);
template <>
__device__ __forceinline__ double2* vecT<double2>(const KArgs& a, int slot, int i) {
  return vec(a, slot, i);
}
template <>
__device__ __forceinline__ float2* vecT<float2>(const KArgs& a, int slot, int i) {
  return a.V32 + ((int64_t)slot * (a.m + 1) + i) * a.ld;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce n complex per-thread values over the workgroup; thread k < n gets value k.
template <int N>
__device__ __forceinline__ double2 block_sum(const double2 (&acc)[N], double2* sh) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double rx = wave_sum(acc[k].x), ry = wave_sum(acc[k].y);
    if (lane == 0) sh[wave * N + k] = make_double2(rx, ry);
  }
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x < N) {
#pragma unroll
    for (int w = 0; w < RBS / 64; ++w) r = cadd(r, sh[w * N + threadIdx.x]);
  }
  __syncthreads();
  return r;
}

// Returns true in exactly one workgroup per slot: the last one to finish.
__device__ __forceinline__ bool last_block(unsigned int* ticket, int nblocks) {
  __shared__ bool is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t = atomicAdd(ticket, 1u);
    is_last = (t == (unsigned)nblocks - 1);
    if (is_last) *ticket = 0;
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last;
}

__device__ __forceinline__ void chunk_range(const KArgs& a, int64_t& b0, int64_t& b1) {
  const int64_t len = (a.ndof + a.nch - 1) / a.nch;
  b0 = (int64_t)blockIdx.x * len;
  b1 = b0 + len < a.ndof ? b0 + len : a.ndof;
}

// Pass 1: h1_i = <hs_i V_i, w>, i <= j, and ||w||^2; pass 2: h2_i = <hs_i V_i, w>.
template <int PASS>
__global__ void __launch_bounds__(RBS) k_dots(KArgs a, int j) {
  __shared__ double2 sh[(RBS / 64) * JB];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  if (st.jstop >= 0) return;
  if (PASS == 2 && st.skip2) return;
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  const double2* __restrict__ w = vec(a, slot, j + 1);
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  for (int g0 = 0; g0 <= j; g0 += JB) {
    double2 acc[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) acc[k] = make_double2(0.0, 0.0);
    const double2* vb[JB];
#pragma unroll
    for (int k = 0; k < JB; ++k) vb[k] = vec(a, slot, (g0 + k <= j) ? g0 + k : 0);
    for (int64_t n = b0 + threadIdx.x; n < b1; n += RBS) {
      const double2 wv = w[n];
#pragma unroll
      for (int k = 0; k < JB; ++k)
        if (g0 + k <= j) {
          const double2 v = vb[k][n];
          acc[k].x += v.x * wv.x + v.y * wv.y;
          acc[k].y += v.x * wv.y - v.y * wv.x;
        }
    }
    const double2 r = block_sum<JB>(acc, sh);
    if (threadIdx.x < JB && g0 + threadIdx.x <= j) part[g0 + threadIdx.x] = r;
  }
  if (PASS == 1) {
    double2 acc1[1] = {make_double2(0.0, 0.0)};
    for (int64_t n = b0 + threadIdx.x; n < b1; n += RBS) {
      const double2 wv = w[n];
      acc1[0].x += wv.x * wv.x + wv.y * wv.y;
    }
    const double2 r = block_sum<1>(acc1, sh);
    if (threadIdx.x == 0) part[MM + 1] = r;
  }
  if (!last_block(&st.ticket[PASS - 1], a.nch)) return;
  const int nv = j + 1 + (PASS == 1 ? 1 : 0);
  for (int i = threadIdx.x; i < nv; i += RBS) {
    const int idx = (i <= j) ? i : MM + 1;
    double2 s = make_double2(0.0, 0.0);
    for (int c = 0; c < a.nch; ++c) s = cadd(s, a.part[((int64_t)slot * a.nch + c) * PSTRIDE + idx]);
    if (i <= j) {
      const double2 h = cscale(s, st.hs[i]);
      if (PASS == 1)
        st.h1[i] = h;
      else
        st.h2[i] = h;
    } else {
      st.nrm0 = sqrt(s.x);
    }
  }
}

// Column j of the Hessenberg matrix (entries 0..j in col, subdiagonal nrm) is final:
// apply the earlier rotations, form the new one, update the residual estimate and
// decide whether the system stops within this cycle. Returns false when the column
// is not finite (the system then stops with the columns before j).
__device__ bool givens_column(SlotState& st, int j, double nrm) {
  double2* col = st.H + (MM + 1) * j;
  double hn2 = nrm * nrm;
  for (int i = 0; i <= j; ++i) hn2 += col[i].x * col[i].x + col[i].y * col[i].y;
  col[j + 1] = make_double2(nrm, 0.0);
  if (!(isfinite(hn2))) {
    st.nonfinite = 1;
    st.jstop = j;
    return false;
  }
  for (int i = 0; i < j; ++i) {
    const double2 a = col[i], b = col[i + 1];
    const double c = st.cs[i];
    const double2 s = st.sn[i];
    col[i] = cadd(cscale(a, c), cmul(s, b));
    col[i + 1] = csub(cscale(b, c), cmulc(s, a));
  }
  const double2 a = col[j];
  const double b = nrm;
  const double aa = hypot(a.x, a.y);
  const double r = hypot(aa, b);
  double c;
  double2 s, rr;
  if (r == 0.0) {
    c = 1.0;
    s = make_double2(0.0, 0.0);
    rr = make_double2(0.0, 0.0);
  } else if (aa == 0.0) {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    rr = make_double2(b, 0.0);
  } else {
    c = aa / r;
    const double2 ph = make_double2(a.x / aa, a.y / aa);
    s = cscale(ph, b / r);
    rr = cscale(ph, r);
  }
  st.cs[j] = c;
  st.sn[j] = s;
  col[j] = rr;
  col[j + 1] = make_double2(0.0, 0.0);
  const double2 g = st.gam[j];
  st.gam[j] = cscale(g, c);
  st.gam[j + 1] = make_double2(-(s.x * g.x + s.y * g.y), -(s.x * g.y - s.y * g.x));  // -conj(s) g
  const double res = hypot(st.gam[j + 1].x, st.gam[j + 1].y);
  const bool breakdown = nrm <= 1e-13 * sqrt(hn2);
  if (res <= fmax(st.tolabs, st.tolcyc) || breakdown) st.jstop = j + 1;
  return true;
}

// Column j from the Gram-Schmidt coefficients (h1, plus h2 after a second pass).
__device__ void finalize_column(SlotState& st, int j, double nrm, bool second) {
  double2* col = st.H + (MM + 1) * j;
  for (int i = 0; i <= j; ++i) col[i] = second ? cadd(st.h1[i], st.h2[i]) : st.h1[i];
  if (!givens_column(st, j, nrm)) {
    st.hs[j + 1] = 0.0;
    return;
  }
  st.hs[j + 1] = (st.jstop < 0 && nrm > 0.0) ? 1.0 / nrm : 0.0;
}

// w -= sum_i (h_i hs_i) V_i and ||w||^2; the last workgroup finalizes.
template <int PASS>
__global__ void __launch_bounds__(RBS) k_update(KArgs a, int j) {
  __shared__ double2 coef[MM + 1];
  __shared__ double2 sh[RBS / 64];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  if (st.jstop >= 0) return;
  if (PASS == 2 && st.skip2) return;
  for (int i = threadIdx.x; i <= j; i += RBS) coef[i] = cscale(PASS == 1 ? st.h1[i] : st.h2[i], st.hs[i]);
  __syncthreads();
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  double2* __restrict__ w = vec(a, slot, j + 1);
  const double2* __restrict__ V0 = vec(a, slot, 0);
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (int64_t n = b0 + threadIdx.x; n < b1; n += RBS) {
    double2 wv = w[n];
    for (int i = 0; i <= j; ++i) {
      const double2 v = V0[(int64_t)i * a.ld + n];
      const double2 c = coef[i];
      wv.x -= c.x * v.x - c.y * v.y;
      wv.y -= c.x * v.y + c.y * v.x;
    }
    w[n] = wv;
    acc[0].x += wv.x * wv.x + wv.y * wv.y;
  }
  const double2 r = block_sum<1>(acc, sh);
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  if (threadIdx.x == 0) part[MM + 1] = r;
  if (!last_block(&st.ticket[2 + PASS - 1], a.nch)) return;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int c = 0; c < a.nch; ++c) s += a.part[((int64_t)slot * a.nch + c) * PSTRIDE + MM + 1].x;
    const double nrm = sqrt(s);
    if (PASS == 1) {
      if (nrm >= 0.7 * st.nrm0 || j + 1 > a.m) {
        st.skip2 = 1;
        finalize_column(st, j, nrm, false);
      } else {
        st.skip2 = 0;
      }
    } else {
      finalize_column(st, j, nrm, true);
    }
  }
}

// First update fused with the second Gram-Schmidt pass: w' = w - sum_i (h1_i hs_i) V_i,
// then h2_i = hs_i <V_i, w'> and ||w'||, with one read of the basis. Each tile of tn
// elements of the chunk is staged in LDS (V_0..V_j and w; the next tile is already in
// flight in registers). The tile width tn is the largest power of two with
// (j+1) tn <= TILE, so a tile stays near 32 KB whatever j is. 256/tn lanes per element
// form w', then lane (i, q) accumulates conj(V_i) w' over a quarter of the tile for
// vectors i, i + 64, ... The last workgroup of a system reduces the chunk partials in a
// fixed order and either keeps h2 for the second update or, when the first pass lost
// less than 30% of the norm, finalizes the column with h1 alone.
constexpr int TILE = 2048;                // staged complex values per tile
constexpr int NDG = (MM + 1 + 63) / 64;   // vector groups of the dot phase
constexpr int VS = TILE + MM + 1 + 64;    // tile with one pad per row (and room for the partials)
__global__ void __launch_bounds__(RBS) k_upd_dots(KArgs a, int j) {
  static_assert((RBS / 64) * (MM + 1) <= VS, "partials reuse the tile buffer");
  __shared__ double2 vs[VS];
  __shared__ double2 wsh[32];
  __shared__ double2 coef[MM + 1];
  __shared__ double nsh[RBS / 64];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  if (st.jstop >= 0) return;
  const int t = threadIdx.x;
  const int nvec = j + 1;
  int tn = 32;
  while (tn > 4 && nvec * tn > TILE) tn >>= 1;
  const int lpe = RBS / tn, tp = tn + 1;
  for (int i = t; i <= j; i += RBS) coef[i] = cscale(st.h1[i], st.hs[i]);
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  double2* __restrict__ w = vec(a, slot, j + 1);
  const double2* __restrict__ V0 = vec(a, slot, 0);
  const int eu = t / lpe, ru = t % lpe;  // update phase: element eu of the tile, part ru
  const int di = t & 63, dq = t >> 6;    // dot phase: vectors di + 64 g; quarter dq of the tile
  const int qlen = tn / 4;
  double2 acc[NDG];
#pragma unroll
  for (int g = 0; g < NDG; ++g) acc[g] = make_double2(0.0, 0.0);
  double nacc = 0.0;
  constexpr int PF = TILE / RBS;
  const int nld = nvec * tn;
  double2 pre[PF], wpre = make_double2(0.0, 0.0);
  auto fetch = [&](int64_t nb) {
    const int len = (int)min((int64_t)tn, b1 - nb);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int q = t + k * RBS, i = q / tn, e = q % tn;
      pre[k] = (q < nld && e < len) ? V0[(int64_t)i * a.ld + nb + e] : make_double2(0.0, 0.0);
    }
    if (t < tn) wpre = t < len ? w[nb + t] : make_double2(0.0, 0.0);
  };
  if (b0 < b1) fetch(b0);
  for (int64_t nb = b0; nb < b1; nb += tn) {
    const int len = (int)min((int64_t)tn, b1 - nb);
    __syncthreads();  // coef ready; previous tile consumed
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      const int q = t + k * RBS;
      if (q < nld) vs[(q / tn) * tp + q % tn] = pre[k];
    }
    if (t < tn) wsh[t] = wpre;
    __syncthreads();
    if (nb + tn < b1) fetch(nb + tn);
    double2 u = make_double2(0.0, 0.0);
    for (int i = ru; i <= j; i += lpe) {
      const double2 v = vs[i * tp + eu], c = coef[i];
      u.x += c.x * v.x - c.y * v.y;
      u.y += c.x * v.y + c.y * v.x;
    }
    for (int o = lpe / 2; o > 0; o >>= 1) {  // groups of lpe lanes are aligned
      u.x += __shfl_xor(u.x, o, 64);
      u.y += __shfl_xor(u.y, o, 64);
    }
    __syncthreads();  // every lane has read wsh's old value
    if (ru == 0) {
      const double2 wn = csub(wsh[eu], u);
      wsh[eu] = wn;
      if (eu < len) {
        w[nb + eu] = wn;
        nacc += wn.x * wn.x + wn.y * wn.y;
      }
    }
    __syncthreads();
    for (int e = dq * qlen; e < (dq + 1) * qlen; ++e) {
      const double2 wv = wsh[e];
#pragma unroll
      for (int g = 0; g < NDG; ++g)
        if (di + 64 * g <= j) {
          const double2 v = vs[(di + 64 * g) * tp + e];
          acc[g].x += v.x * wv.x + v.y * wv.y;
          acc[g].y += v.x * wv.y - v.y * wv.x;
        }
    }
  }
  // block partials (in the tile buffer): h2 sums over the quarters, ||w'||^2 over the waves
  double2* red = vs;  // [RBS/64][MM+1]
  const double nw = wave_sum(nacc);
  __syncthreads();
#pragma unroll
  for (int g = 0; g < NDG; ++g)
    if (di + 64 * g <= j) red[dq * (MM + 1) + di + 64 * g] = acc[g];
  if ((t & 63) == 0) nsh[t >> 6] = nw;
  __syncthreads();
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  for (int i = t; i <= j; i += RBS) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < RBS / 64; ++q) sum = cadd(sum, red[q * (MM + 1) + i]);
    part[i] = sum;
  }
  if (t == 0) {
    double sn = 0.0;
#pragma unroll
    for (int q = 0; q < RBS / 64; ++q) sn += nsh[q];
    part[MM + 1] = make_double2(sn, 0.0);
  }
  if (!last_block(&st.ticket[2], a.nch)) return;
  __shared__ double nrm_sh;
  if (t == 0) {
    double sn = 0.0;
    for (int c = 0; c < a.nch; ++c) sn += a.part[((int64_t)slot * a.nch + c) * PSTRIDE + MM + 1].x;
    nrm_sh = sqrt(sn);
  }
  __syncthreads();
  const double nrm = nrm_sh;
  const bool skip = nrm >= 0.7 * st.nrm0 || j + 1 > a.m;
  if (!skip) {
    for (int i = t; i <= j; i += RBS) {
      double2 sum = make_double2(0.0, 0.0);
      for (int c = 0; c < a.nch; ++c) sum = cadd(sum, a.part[((int64_t)slot * a.nch + c) * PSTRIDE + i]);
      st.h2[i] = cscale(sum, st.hs[i]);
    }
  }
  if (t == 0) {
    st.skip2 = skip ? 1 : 0;
    if (skip) finalize_column(st, j, nrm, false);
  }
}

// ---- Lagged classical Gram-Schmidt with reorthogonalization (DCGS2) ----
// (Swirydowicz, Langou, Ananthan, Yang, Thomas, 2020.) Step j starts from
// u = hs_j V_j, orthogonalized once against q_0..q_{j-1}, and W = A P^-1 u in V_{j+1}.
// Pass 1 (k_lag_dots) forms S_i = <V_i, V_j> and A_i = <V_i, W>, i <= j, in one read.
// Its last workgroup then
//   * reorthogonalizes u on paper: s_i = <q_i, u>, sigma^2 = |u|^2 - |s|^2, so that
//     u = Q s + sigma q_j, and completes column j-1 (its first-pass part plus rho s,
//     subdiagonal rho sigma, rho being |u|'s first-pass norm) and its Givens rotation;
//   * derives the projections of A P^-1 q_j = (W - [Q q_j] H s) / sigma without touching
//     the vectors: with a_i = <q_i, W> and gamma = <q_j, W> = (<u, W> - s^H a) / sigma,
//     column j's first-pass part is ([a; gamma] - H s) / sigma.
// Pass 2 (k_lag_update) writes q_j = (u - Q s) / sigma over V_j and the next first-pass
// vector (W - Q a - gamma q_j) / sigma over V_{j+1}, sharing one read of the basis, and
// its norm rho_j. After the last step one more pass 1 (final) completes the last column.
constexpr int VS2 = (RBS / 64) * 2 * (MM + 1);  // per-wavefront partials, then the final sums
template <class VT>
__global__ void __launch_bounds__(RBS) k_lag_dots(KArgs a, int j, int final) {
  __shared__ double2 vsd[VS2];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  if (st.jstop >= 0) return;
  const int t = threadIdx.x;
  // each wavefront streams runs of 64 * E consecutive values of u = V_j, W and every
  // V_i (as pass 2 does); per vector the lane sums of conj(V_i) u and conj(V_i) W are
  // reduced across the wavefront and added to the wavefront's partials in LDS, which
  // are summed over the wavefronts in a fixed order
  constexpr int E = 16;
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  const VT* __restrict__ V0 = vecT<VT>(a, slot, 0);
  const int lane = t & 63, wave = t >> 6;
  double2* red = vsd;  // [RBS/64][2(MM+1)]
  const int R2 = 2 * (MM + 1);
  for (int i = lane; i < 2 * (j + 1); i += 64) red[wave * R2 + i] = make_double2(0.0, 0.0);
  for (int64_t nb = b0 + (int64_t)wave * 64 * E; nb < b1; nb += (int64_t)RBS * E) {
    double2 uv[E], wv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t n = nb + lane + 64 * e;
      uv[e] = n < b1 ? to_d2(V0[(int64_t)j * a.ld + n]) : make_double2(0.0, 0.0);
      wv[e] = (n < b1 && !final) ? to_d2(V0[(int64_t)(j + 1) * a.ld + n]) : make_double2(0.0, 0.0);
    }
    for (int i = 0; i <= j; ++i) {
      const VT* __restrict__ vi = V0 + (int64_t)i * a.ld;
      double sx = 0.0, sy = 0.0, ax = 0.0, ay = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t n = nb + lane + 64 * e;
        const double2 v = n < b1 ? to_d2(vi[n]) : make_double2(0.0, 0.0);
        sx += v.x * uv[e].x + v.y * uv[e].y;
        sy += v.x * uv[e].y - v.y * uv[e].x;
        ax += v.x * wv[e].x + v.y * wv[e].y;
        ay += v.x * wv[e].y - v.y * wv[e].x;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_xor(sx, o);
        sy += __shfl_xor(sy, o);
        ax += __shfl_xor(ax, o);
        ay += __shfl_xor(ay, o);
      }
      if (lane == 0) {
        double2& rs = red[wave * R2 + 2 * i];
        double2& ra = red[wave * R2 + 2 * i + 1];
        rs.x += sx;
        rs.y += sy;
        ra.x += ax;
        ra.y += ay;
      }
    }
  }
  __syncthreads();
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  for (int i = t; i < 2 * (j + 1); i += RBS) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < RBS / 64; ++q) sum = cadd(sum, red[q * R2 + i]);
    part[i] = sum;
  }
  if (!last_block(&st.ticket[0], a.nch)) return;
  // ---- last workgroup: fixed-order sums over the chunks, then the scalar work ----
  double2* S = vsd;            // [MM+1]
  double2* Av = vsd + MM + 1;  // [MM+1]
  __shared__ double sh_sig, sh_rho;
  __shared__ int sh_go;
  for (int i = t; i <= j; i += RBS) {
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    for (int c = 0; c < a.nch; ++c) {
      const double2* pc = a.part + ((int64_t)slot * a.nch + c) * PSTRIDE;
      s0 = cadd(s0, pc[2 * i]);
      s1 = cadd(s1, pc[2 * i + 1]);
    }
    S[i] = s0;
    Av[i] = s1;
  }
  __syncthreads();
  const double hsj = st.hs[j];
  // s_i = <q_i, u> (i < j) into h1, a_i = <q_i, W> into h2
  for (int i = t; i < j; i += RBS) {
    st.h1[i] = cscale(S[i], st.hs[i] * hsj);
    if (!final) st.h2[i] = cscale(Av[i], st.hs[i]);
  }
  __syncthreads();
  if (t == 0) {
    double ss = 0.0;
    for (int i = 0; i < j; ++i) ss += st.h1[i].x * st.h1[i].x + st.h1[i].y * st.h1[i].y;
    const double nu = hsj * hsj * S[j].x;
    const double sg2 = nu - ss;
    const double sig = sg2 > 1e-28 * nu ? sqrt(sg2) : 0.0;
    sh_sig = sig;
    sh_rho = st.rho;
    sh_go = 1;
  }
  __syncthreads();
  const double sig = sh_sig, rho = sh_rho;
  if (j > 0) {
    // complete column j-1 and rotate it
    double2* hu = st.Hu + (MM + 1) * (j - 1);
    for (int i = t; i < j; i += RBS) hu[i] = cadd(hu[i], cscale(st.h1[i], rho));
    __syncthreads();
    if (t == 0) {
      hu[j] = make_double2(rho * sig, 0.0);
      double2* col = st.H + (MM + 1) * (j - 1);
      for (int i = 0; i < j; ++i) col[i] = hu[i];
      givens_column(st, j - 1, rho * sig);
      if (st.jstop >= 0 || final || !(sig > 0.0)) {
        if (st.jstop < 0) st.jstop = j;  // u in the span of Q: the space is invariant
        sh_go = 0;
      }
    }
    __syncthreads();
  } else if (t == 0 && !(sig > 0.0)) {
    st.jstop = 0;
    sh_go = 0;
  }
  if (final) return;
  __syncthreads();
  if (!sh_go) return;
  // gamma = (<u, W> - s^H a) / sigma, then column j's first-pass part ([a; gamma] - H s) / sigma
  __shared__ double2 sh_g;
  if (t == 0) {
    double2 g = cscale(Av[j], hsj);
    for (int i = 0; i < j; ++i) {
      const double2 si = st.h1[i], ai = st.h2[i];
      g.x -= si.x * ai.x + si.y * ai.y;
      g.y -= si.x * ai.y - si.y * ai.x;
    }
    g = cscale(g, 1.0 / sig);
    sh_g = g;
    st.gq = g;
    st.sig = sig;
  }
  __syncthreads();
  double2* huj = st.Hu + (MM + 1) * j;
  for (int r = t; r <= j; r += RBS) {
    double2 c = r < j ? st.h2[r] : sh_g;
    for (int i = (r > 0 ? r - 1 : 0); i < j; ++i) c = csub(c, cmul(st.Hu[(MM + 1) * i + r], st.h1[i]));
    huj[r] = cscale(c, 1.0 / sig);
  }
}

// Pass 2 of a lagged step: q_j over V_j, the next first-pass vector over V_{j+1}, and its norm.
template <class VT>
__global__ void __launch_bounds__(RBS) k_lag_update(KArgs a, int j) {
  __shared__ double2 cq[MM + 1], cw[MM + 1];
  __shared__ double2 sh[RBS / 64];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  if (st.jstop >= 0) return;
  for (int i = threadIdx.x; i < j; i += RBS) {
    cq[i] = cscale(st.h1[i], st.hs[i]);
    cw[i] = cscale(st.h2[i], st.hs[i]);
  }
  __syncthreads();
  const double hsj = st.hs[j], inv = 1.0 / st.sig;
  const double2 gq = st.gq;
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  VT* __restrict__ u = vecT<VT>(a, slot, j);
  VT* __restrict__ w = vecT<VT>(a, slot, j + 1);
  const VT* __restrict__ V0 = vecT<VT>(a, slot, 0);
  double2 acc[1] = {make_double2(0.0, 0.0)};
  // each wavefront takes E * 64 consecutive elements, so every basis vector is read in
  // runs of E * 64 values (longer DRAM bursts than one value per lane per vector)
  constexpr int E = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t nb = b0 + (int64_t)wave * 64 * E; nb < b1; nb += (int64_t)RBS * E) {
    double2 sq[E], sw[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sq[e] = sw[e] = make_double2(0.0, 0.0);
#pragma unroll 2
    for (int i = 0; i < j; ++i) {
      const VT* __restrict__ vi = V0 + (int64_t)i * a.ld;
      double2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t n = nb + lane + 64 * e;
        v[e] = n < b1 ? to_d2(vi[n]) : make_double2(0.0, 0.0);
      }
      const double2 ci = cq[i], wi = cw[i];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        sq[e] = cadd(sq[e], cmul(ci, v[e]));
        sw[e] = cadd(sw[e], cmul(wi, v[e]));
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t n = nb + lane + 64 * e;
      if (n < b1) {
        const double2 uv = to_d2(u[n]), wv = to_d2(w[n]);
        const double2 q = cscale(csub(cscale(uv, hsj), sq[e]), inv);
        const double2 wn = cscale(csub(csub(wv, sw[e]), cmul(gq, q)), inv);
        u[n] = cvt2<VT>(q);
        w[n] = cvt2<VT>(wn);
        acc[0].x += wn.x * wn.x + wn.y * wn.y;
      }
    }
  }
  const double2 r = block_sum<1>(acc, sh);
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  if (threadIdx.x == 0) part[MM + 1] = r;
  if (!last_block(&st.ticket[1], a.nch)) return;
  if (threadIdx.x == 0) {
    double sn = 0.0;
    for (int c = 0; c < a.nch; ++c) sn += a.part[((int64_t)slot * a.nch + c) * PSTRIDE + MM + 1].x;
    const double rho = sqrt(sn);
    st.hs[j] = 1.0;
    double2* huj = st.Hu + (MM + 1) * j;
    double hn2 = 0.0;
    for (int i = 0; i <= j; ++i) hn2 += huj[i].x * huj[i].x + huj[i].y * huj[i].y;
    if (!(rho > 1e-13 * sqrt(hn2)) || !isfinite(rho)) {
      // the new direction vanished: column j is final with a zero subdiagonal
      double2* col = st.H + (MM + 1) * j;
      for (int i = 0; i <= j; ++i) col[i] = huj[i];
      givens_column(st, j, 0.0);
      if (st.jstop < 0) st.jstop = j + 1;
      st.hs[j + 1] = 0.0;
      st.rho = 0.0;
    } else {
      st.rho = rho;
      st.hs[j + 1] = 1.0 / rho;
      huj[j + 1] = make_double2(rho, 0.0);
    }
  }
}

// Back substitution R y = gamma over the steps of this cycle; y_i *= hs_i.
__global__ void k_trisolve(KArgs a, int nact) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  const int slot = a.act[k];
  SlotState& st = a.st[slot];
  const int J = st.jstop >= 0 ? st.jstop : a.m;
  for (int i = J - 1; i >= 0; --i) {
    double2 s = st.gam[i];
    for (int l = i + 1; l < J; ++l) s = csub(s, cmul(st.H[(MM + 1) * l + i], st.y[l]));
    const double2 d = st.H[(MM + 1) * i + i];
    const double dn = d.x * d.x + d.y * d.y;
    st.y[i] = dn > 0.0 ? make_double2((s.x * d.x + s.y * d.y) / dn, (s.y * d.x - s.x * d.y) / dn)
                       : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < J; ++i) st.y[i] = cscale(st.y[i], st.hs[i]);
  st.lastJ = J;
}

// t = sum_{i<J} y_i V_i
template <class VT>
__global__ void __launch_bounds__(RBS) k_combine(KArgs a, VArg t) {
  __shared__ double2 y[MM];
  const int slot = a.act[blockIdx.y];
  const SlotState& st = a.st[slot];
  const int J = st.lastJ;
  for (int i = threadIdx.x; i < J; i += RBS) y[i] = st.y[i];
  __syncthreads();
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  const VT* __restrict__ V0 = vecT<VT>(a, slot, 0);
  double2* __restrict__ ts = t.at(slot);
  for (int64_t n = b0 + threadIdx.x; n < b1; n += RBS) {
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < J; ++i) {
      const double2 v = to_d2(V0[(int64_t)i * a.ld + n]);
      s.x += y[i].x * v.x - y[i].y * v.y;
      s.y += y[i].x * v.y + y[i].y * v.x;
    }
    ts[n] = s;
  }
}

// Mixed precision: x += z with the velocity part from the FP32 vector and the
// pressure part from the FP64 Schur-block result.
__global__ void k_axpy32(KArgs a, VArg x, VArg32 z, VArg zp, int64_t DN) {
  const int slot = a.act[blockIdx.y];
  double2* xs = x.at(slot);
  const float2* zs = z.at(slot);
  const double2* zps = zp.at(slot);
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.ndof; n += (int64_t)gridDim.x * blockDim.x) {
    if (n < DN) {
      const float2 zv = zs[n];
      xs[n] = make_double2(xs[n].x + (double)zv.x, xs[n].y + (double)zv.y);
    } else {
      xs[n] = cadd(xs[n], zps[n]);
    }
  }
}

__global__ void k_axpy(KArgs a, VArg x, VArg z) {
  const int slot = a.act[blockIdx.y];
  double2* xs = x.at(slot);
  const double2* zs = z.at(slot);
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.ndof; n += (int64_t)gridDim.x * blockDim.x)
    xs[n] = cadd(xs[n], zs[n]);
}

// ||x||: KIND 0 sets fnorm/tolabs from the right-hand side; KIND 1 starts a
// cycle from the residual stored in V_0.
// KIND 0: ||f|| and the absolute target; KIND 1: ||r|| of the current iterate, which
// starts a cycle (with `inner` > 0 the cycle also ends once its own residual estimate
// has fallen by that factor, as inner solves of iterative refinement do).
template <int KIND, class VT = double2>
__global__ void __launch_bounds__(RBS) k_norm(KArgs a, VArg x, double rtol, double inner = 0.0) {
  __shared__ double2 sh[RBS / 64];
  const int slot = a.act[blockIdx.y];
  SlotState& st = a.st[slot];
  int64_t b0, b1;
  chunk_range(a, b0, b1);
  const double2* __restrict__ xs = x.at(slot);
  const VT* __restrict__ v0 = vecT<VT>(a, slot, 0);
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (int64_t n = b0 + threadIdx.x; n < b1; n += RBS) {
    const double2 v = KIND == 0 ? xs[n] : to_d2(v0[n]);
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  const double2 r = block_sum<1>(acc, sh);
  double2* part = a.part + ((int64_t)slot * a.nch + blockIdx.x) * PSTRIDE;
  if (threadIdx.x == 0) part[MM + 1] = r;
  if (!last_block(&st.ticket[4 + KIND], a.nch)) return;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int c = 0; c < a.nch; ++c) s += a.part[((int64_t)slot * a.nch + c) * PSTRIDE + MM + 1].x;
    const double nrm = sqrt(s);
    if (KIND == 0) {
      st.fnorm = nrm;
      st.tolabs = rtol * nrm;
      st.nonfinite = isfinite(nrm) ? 0 : 1;
    } else {
      st.beta = nrm;
      st.tolcyc = inner * nrm;
      st.gam[0] = make_double2(nrm, 0.0);
      st.hs[0] = nrm > 0.0 ? 1.0 / nrm : 0.0;
      st.jstop = (nrm <= st.tolabs || !isfinite(nrm)) ? 0 : -1;
      st.skip2 = 1;
      if (!isfinite(nrm)) st.nonfinite = 1;
      double* inf = a.info + 4 * slot;
      inf[0] = st.fnorm > 0.0 ? nrm / st.fnorm : nrm;
      inf[1] = st.lastJ;
      inf[2] = st.nonfinite;
      inf[3] = nrm;
    }
  }
}

// x = x0 (or 0) with the Dirichlet data written into the constrained rows.
template <int D>
__global__ void k_init_x(VArg x, const double2* __restrict__ x0, int64_t x0st, const double2* __restrict__ g,
                         int64_t gst, const int32_t* __restrict__ dmask, const int32_t* __restrict__ dirnodes,
                         int64_t ndir, int64_t n2, int64_t ndof, const int* act, int first) {
  const int slot = act[blockIdx.y];
  const int sys = first + slot;  // slot k of a batch holds system first + k
  double2* xs = x.at(slot);
  // Entries of Dirichlet (kind 2) nodes are written only by the second loop
  // when data is given, so the two loops never write the same element.
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < ndof; n += (int64_t)gridDim.x * blockDim.x) {
    double2 v = x0 ? x0[(int64_t)sys * x0st + n] : make_double2(0.0, 0.0);
    const int32_t dm = n < D * n2 ? dmask[n / D] : 0;
    if (dm == 2 && g) continue;
    if (dm != 0) v = make_double2(0.0, 0.0);
    xs[n] = v;
  }
  if (!g) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndir * D;
       i += (int64_t)gridDim.x * blockDim.x)
    xs[(int64_t)dirnodes[i / D] * D + (i % D)] = g[(int64_t)sys * gst + i];
}

// a[idx[k]] = 0 for the listed slots (a fill kernel: no memset node in captured work)
__global__ void k_zero_at(double* a, const int* idx, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[idx[k]] = 0.0;
}

__global__ void k_init_state(SlotState* st, const int* act, int nact) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nact) return;
  SlotState& s = st[act[k]];
  for (int i = 0; i < 8; ++i) s.ticket[i] = 0;
  s.jstop = -1;
  s.skip2 = 1;
  s.nonfinite = 0;
  s.lastJ = 0;
  for (int i = 0; i <= MM; ++i) s.hs[i] = 0.0;
}

__global__ void k_copy_out(const VArg x, const int* act, int first, int nact, int64_t n2, int D, int64_t nv,
                           double2* __restrict__ u, double2* __restrict__ p) {
  const int k = blockIdx.y;
  const int slot = act[k];
  const int64_t sys = first + k;
  const double2* xs = x.at(slot);
  const int64_t DN = (int64_t)D * n2;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < DN + nv; n += (int64_t)gridDim.x * blockDim.x) {
    if (n < DN)
      u[sys * DN + n] = xs[n];
    else
      p[sys * nv + (n - DN)] = xs[n];
  }
}

// Device workspace for a batch of `slots` systems.
struct Pool {
  int slots = 0, m = 0, nch = 0;
  bool v32 = false;  // Krylov basis stored as FP32 pairs (arithmetic stays FP64)
  int64_t ld = 0, DN = 0, nv = 0;
  DBuf<double2> V, W, vt, pt, part, trac;
  DBuf<float2> vt32, z32;
  DBuf<SlotState> st;
  DBuf<double> omega, lv, info;
  DBuf<int> act, act_all, act_run, act_new, stops;
  DBuf<double2> zil;  // interleaved preconditioner output inside a cycle (FP32 pairs in mixed mode)
  DBuf<char> mgbuf;   // multigrid temporaries below level 0
  DBuf<double> mglam; // [velocity level][slot] smoother bounds
  DBuf<double2> mginv; // [slot] dense inverse of the coarsest velocity level
  DBuf<float2> mginv32;
  VArg Z() const { return VArg{W.p, 4 * ld}; }
  VArg X() const { return VArg{W.p + ld, 4 * ld}; }
  VArg F() const { return VArg{W.p + 2 * ld, 4 * ld}; }
  VArg T() const { return VArg{W.p + 3 * ld, 4 * ld}; }
};

size_t slot_bytes(int64_t ld, int m, int64_t DN, int64_t nv, int nch, bool mixed, bool v32) {
  // basis, Z/X/F/T, velocity temps (FP64 path), pressure temps, partial sums; FP32 temps,
  // z32 (mixed path); interleaved operator input (FP32 pairs in mixed mode)
  return (v32 ? sizeof(float2) : sizeof(double2)) * (size_t)(m + 1) * ld +
         sizeof(double2) * ((size_t)4 * ld + (mixed ? 0 : 4 * DN) + 4 * nv + (size_t)nch * PSTRIDE) +
         (mixed ? sizeof(float2) * (4 * DN + ld) : 0) + (mixed ? sizeof(float2) : sizeof(double2)) * ld +
         sizeof(SlotState) + 64;
}

int choose_nch(int nact, int64_t ndof) {
  int nch = (2048 + nact - 1) / nact;
  const int64_t maxc = (ndof + RBS - 1) / RBS;
  if (nch > maxc) nch = (int)maxc;
  return nch < 1 ? 1 : nch;
}

KArgs kargs(Pool& P, int64_t ndof, int nch) {
  KArgs a;
  a.act = P.act;
  a.st = P.st;
  a.part = P.part;
  a.nch = nch;
  a.ndof = ndof;
  a.ld = P.ld;
  a.m = P.m;
  a.V = P.V;
  a.V32 = reinterpret_cast<float2*>(P.V.p);
  a.info = P.info;
  return a;
}

// Steps j0..j1-1 of a restart cycle for the systems of `br` that are still running
// (a system that stops inside the chunk makes its later Arnoldi launches return at once).
void cycle_steps(scvs_mesh m, Pool& P, const Batch& br, const PrecondArgs& pa, int64_t ndof, int j0, int j1,
                 bool lagged, hipStream_t s) {
  const int nact = br.nact;
  const int nch = choose_nch(nact, ndof);
  KArgs a = kargs(P, ndof, nch);
  a.act = br.act;
  const dim3 gr((unsigned)nch, (unsigned)nact);
  const int64_t vst = (int64_t)(P.m + 1) * P.ld;
  Profiler* prof = &m->ctx->prof;
  // one basis vector of every running system
  const double vec = (double)ndof * (P.v32 ? 8.0 : 16.0) * nact;
  for (int j = j0; j < j1; ++j) {
    Batch bj = br;
    bj.insc = reinterpret_cast<const double*>(P.st.p) + offsetof(SlotState, hs) / sizeof(double) + j;
    bj.insc_st = sizeof(SlotState) / sizeof(double);
    bj.insc_idx = 0;
    if (P.v32) {
      float2* V32 = reinterpret_cast<float2*>(P.V.p);
      precond_apply(m, bj, pa, VArg32{V32 + (int64_t)j * P.ld, vst}, P.Z(), s, P.zil.p);
      spmv_apply_il(m, br, P.zil.p, pa.mixed != 0, VArg32{V32 + (int64_t)(j + 1) * P.ld, vst}, s);
    } else {
      precond_apply(m, bj, pa, VArg{P.V.p + (int64_t)j * P.ld, vst}, P.Z(), s, P.zil.p);
      spmv_apply_il(m, br, P.zil.p, pa.mixed != 0, VArg{P.V.p + (int64_t)(j + 1) * P.ld, vst}, s);
    }
    if (lagged) {
      {
        ProfScope ps(prof, s, "k_lag_dots", vec * (j + 2));  // V_0..V_j and W once
        if (P.v32)
          k_lag_dots<float2><<<gr, RBS, 0, s>>>(a, j, 0);
        else
          k_lag_dots<double2><<<gr, RBS, 0, s>>>(a, j, 0);
      }
      {
        ProfScope ps(prof, s, "k_lag_update", vec * (j + 4));  // V_0..V_j and W read, V_j and W written
        if (P.v32)
          k_lag_update<float2><<<gr, RBS, 0, s>>>(a, j);
        else
          k_lag_update<double2><<<gr, RBS, 0, s>>>(a, j);
      }
    } else {
      {
        ProfScope ps(prof, s, "k_dots1", vec * (j + 2));  // V_0..V_j and w once
        k_dots<1><<<gr, RBS, 0, s>>>(a, j);
      }
      {
        ProfScope ps(prof, s, "k_upd_dots", vec * (j + 3));  // V_0..V_j and w read, w written
        k_upd_dots<<<gr, RBS, 0, s>>>(a, j);
      }
      {
        ProfScope ps(prof, s, "k_update2", vec * (j + 3));
        k_update<2><<<gr, RBS, 0, s>>>(a, j);
      }
    }
    launch_check(s);
  }
}

__global__ void k_stops(const SlotState* __restrict__ st, const int* __restrict__ act, int n, int* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = st[act[k]].jstop;
}

// End of a restart cycle for the systems of `b` (all that started it): least squares,
// x += P^-1 V y, and the new true residual.
void cycle_end(scvs_mesh m, Pool& P, const Batch& b, const PrecondArgs& pa, int64_t ndof, double rtol,
               double inner, bool lagged, hipStream_t s) {
  const int nact = b.nact;
  const int nch = choose_nch(nact, ndof);
  KArgs a = kargs(P, ndof, nch);
  a.act = b.act;
  const dim3 gr((unsigned)nch, (unsigned)nact);
  const int64_t vst = (int64_t)(P.m + 1) * P.ld;
  Profiler* prof = &m->ctx->prof;
  const double vec = (double)ndof * 16.0 * nact;
  const double vecb = (double)ndof * (P.v32 ? 8.0 : 16.0) * nact;  // one basis vector of each
  if (lagged) {
    // the last column still needs the lagged correction of V_m
    ProfScope ps(prof, s, "k_lag_dots", vecb * (P.m + 1));
    if (P.v32)
      k_lag_dots<float2><<<gr, RBS, 0, s>>>(a, P.m, 1);
    else
      k_lag_dots<double2><<<gr, RBS, 0, s>>>(a, P.m, 1);
  }
  {
    ProfScope ps(prof, s, "k_trisolve", 0.0);
    k_trisolve<<<(nact + 63) / 64, 64, 0, s>>>(a, nact);
  }
  {
    ProfScope ps(prof, s, "k_combine", vecb * P.m + vec);
    if (P.v32)
      k_combine<float2><<<gr, RBS, 0, s>>>(a, P.T());
    else
      k_combine<double2><<<gr, RBS, 0, s>>>(a, P.T());
  }
  precond_apply(m, b, pa, P.T(), P.Z(), s);
  {
    ProfScope ps(prof, s, "k_axpy", vec * (pa.mixed ? 2.5 : 3.0));
    if (pa.mixed)
      k_axpy32<<<dim3(256, nact), 256, 0, s>>>(a, P.X(), pa.z32, P.Z(), P.DN);
    else
      k_axpy<<<dim3(256, nact), 256, 0, s>>>(a, P.X(), P.Z());
  }
  if (P.v32)
    spmv_resid32(m, b, P.X(), VArg32{reinterpret_cast<float2*>(P.V.p), vst}, P.F(), s, P.T());
  else
    spmv_full(m, b, P.X(), VArg{P.V.p, vst}, SPMV_RESID, true, P.F(), nullptr, s);
  {
    ProfScope ps(prof, s, "k_norm", vecb);
    if (P.v32)
      k_norm<1, float2><<<gr, RBS, 0, s>>>(a, VArg{}, rtol, pa.mixed ? inner : 0.0);
    else
      k_norm<1, double2><<<gr, RBS, 0, s>>>(a, VArg{}, rtol, pa.mixed ? inner : 0.0);
  }
  launch_check(s);
}

}  // namespace

void scatter_dirichlet(scvs_mesh m, int64_t nsys, const void* g, VArg x, const int* act, hipStream_t s) {
  const int D = m->dim;
  const int64_t ndof = D * m->n2 + m->nv;
  const dim3 gi(256, (unsigned)nsys);
  const double2* gp = (const double2*)g;
  if (D == 2)
    k_init_x<2><<<gi, 256, 0, s>>>(x, nullptr, 0, gp, m->ndir * D, m->dmask, m->dirnodes, m->ndir, m->n2, ndof, act,
                                   0);
  else
    k_init_x<3><<<gi, 256, 0, s>>>(x, nullptr, 0, gp, m->ndir * D, m->dmask, m->dirnodes, m->ndir, m->n2, ndof, act,
                                   0);
  launch_check(s);
}

void rhs_systems(scvs_mesh m, int64_t nsys, const double* omega, const double* traction, const void* g, void* f) {
  hipStream_t s = m->ctx->stream;
  const int D = m->dim;
  const int64_t ndof = D * m->n2 + m->nv;
  const int ntr = (int)m->traction_tags.size();
  DBuf<double> om;
  DBuf<double2> tr, xg;
  DBuf<int> act;
  std::vector<int> acth(nsys);
  for (int64_t k = 0; k < nsys; ++k) acth[k] = (int)k;
  om.upload(omega, nsys, s);
  tr.alloc((size_t)nsys * std::max(ntr, 1));
  if (ntr) SCVS_HIP(hipMemcpyAsync(tr.p, traction, sizeof(double2) * nsys * ntr, hipMemcpyHostToDevice, s));
  act.upload(acth.data(), nsys, s);
  xg.alloc((size_t)nsys * ndof);
  const dim3 gi(256, (unsigned)nsys);
  if (D == 2)
    k_init_x<2><<<gi, 256, 0, s>>>(VArg{xg.p, ndof}, nullptr, 0, (const double2*)g, m->ndir * D, m->dmask,
                                   m->dirnodes, m->ndir, m->n2, ndof, act, 0);
  else
    k_init_x<3><<<gi, 256, 0, s>>>(VArg{xg.p, ndof}, nullptr, 0, (const double2*)g, m->ndir * D, m->dmask,
                                   m->dirnodes, m->ndir, m->n2, ndof, act, 0);
  launch_check(s);
  Batch b;
  b.nact = (int)nsys;
  b.act = act;
  b.omega = om;
  spmv_full(m, b, VArg{xg.p, ndof}, VArg{(double2*)f, ndof}, SPMV_RHS, false, VArg{}, tr, s);
  SCVS_HIP(hipStreamSynchronize(s));
}

int solve_systems(scvs_mesh m, int64_t nsys, const double* omega, const double* traction, const void* g,
                  const void* x0, void* u_out, void* p_out, const scvs_solve_opts* o, scvs_report* rep) {
  hipStream_t s = m->ctx->stream;
  const int D = m->dim;
  const int64_t ndof = D * m->n2 + m->nv;
  const int64_t DN = D * m->n2;
  const int ntr = (int)m->traction_tags.size();
  Pool P;
  P.ld = (ndof + 63) / 64 * 64;
  P.DN = DN;
  P.nv = m->nv;
  // batch size from free memory (keep 10% spare), or from the context's memory cap if that
  // is smaller; a long restart that would leave room for fewer than min(nsys, 8) systems
  // is shortened (not below 30) first
  size_t fr = 0, tot = 0;
  SCVS_HIP(hipMemGetInfo(&fr, &tot));
  const int nch_max = choose_nch(1, ndof);
  const bool mixed = o->precision >= 1;
  const bool lagged = o->orth == 1;
  P.v32 = o->precision == 2;  // FP32 basis storage (lagged orthogonalization only; checked by the caller)
  if (mixed) {
    make_fp32_copies(m, s);
    s2sell_setup(m, true, false, s);  // the operator product reads S2 in sliced rows
  }
  // multigrid blocks: the hierarchy (once per assembly and boundary conditions) and, per
  // slot, a fifth level-0 temporary, the coarse-level temporaries and the smoother bounds
  const bool vmg = o->vel_block == 1, pmg = o->pres_block == 1 && o->cheb_pres > 0;
  const size_t esz = mixed ? sizeof(float2) : sizeof(double2);
  size_t mg_extra = 0;
  if (vmg || pmg) {
    mg_setup(m, s);
    mg_sell_values(m, mixed, vmg, pmg, s);
    const size_t nc2 = (size_t)mg_coarse_rows(m) * mg_coarse_rows(m);
    mg_extra = (vmg ? (size_t)DN * esz + nc2 * (sizeof(double2) + (mixed ? sizeof(float2) : 0)) : 0) +
               (pmg ? (size_t)m->nv * sizeof(double2) : 0) + mg_buffer_bytes(m, 1, esz, vmg, pmg) +
               sizeof(double) * mg_levels(m, true);
  }
  double budget = (double)fr * 0.9;
  if (m->ctx->mem_cap > 0) budget = std::min(budget, (double)m->ctx->mem_cap);
  int mk = o->restart;
  const int64_t want = std::min<int64_t>(nsys, 8);
  while (mk > 30 &&
         (int64_t)(budget / (double)(slot_bytes(P.ld, mk, DN, m->nv, nch_max, mixed, P.v32) + mg_extra)) < want)
    mk = std::max(30, mk * 3 / 4);
  if (o->verbose && mk != o->restart) fprintf(stderr, "[scvs] restart shortened to %d to fit memory\n", mk);
  P.m = mk;
  const size_t per = slot_bytes(P.ld, mk, DN, m->nv, nch_max, mixed, P.v32) + mg_extra;
  int64_t fit = (int64_t)(budget / (double)per);
  SCVS_REQUIRE(fit >= 1, SCVS_E_NOMEM,
               "not enough device memory (or memory cap) for one system's Krylov workspace of " +
                   std::to_string(per) + " bytes");
  int B = (int)std::min<int64_t>(nsys, fit);
  if (o->max_batch > 0) B = std::min(B, o->max_batch);
  if (o->verbose)
    fprintf(stderr, "[scvs] slot pool: %d slots of %zu bytes (budget %.0f bytes)\n", B, per, budget);
  P.slots = B;
  P.V.alloc(P.v32 ? ((size_t)B * (mk + 1) * P.ld + 1) / 2 : (size_t)B * (mk + 1) * P.ld);
  P.W.alloc((size_t)B * 4 * P.ld);
  const int nvt = vmg ? 5 : 4, npt = pmg ? 5 : 4;
  if (mixed) {
    P.vt32.alloc((size_t)B * nvt * DN);
    P.z32.alloc((size_t)B * P.ld);
  } else {
    P.vt.alloc((size_t)B * nvt * DN);
  }
  P.pt.alloc((size_t)B * npt * m->nv);
  if (vmg || pmg) {
    P.mgbuf.alloc(mg_buffer_bytes(m, B, esz, vmg, pmg) + 256);
    P.mglam.alloc((size_t)B * mg_levels(m, true));
    if (vmg) {
      const size_t nc2 = (size_t)mg_coarse_rows(m) * mg_coarse_rows(m);
      P.mginv.alloc((size_t)B * nc2);
      if (mixed) P.mginv32.alloc((size_t)B * nc2);
    }
  }
  P.part.alloc((size_t)B * nch_max * PSTRIDE);
  P.st.alloc(B);
  P.omega.alloc(B);
  P.lv.alloc(B);
  P.info.alloc(4 * B);
  P.act.alloc(B);
  P.act_all.alloc(B);
  P.act_run.alloc(B);
  P.stops.alloc(B);
  P.zil.alloc(mixed ? ((size_t)B * P.ld + 1) / 2 : (size_t)B * P.ld);
  P.trac.alloc((size_t)B * std::max(ntr, 1));
  PrecondArgs pa;
  pa.kv = o->cheb_vel;
  pa.kp = o->cheb_pres;
  pa.ratio = o->cheb_ratio;
  pa.ratio_p = o->cheb_ratio_pres > 0.0 ? o->cheb_ratio_pres : o->cheb_ratio;
  pa.vt = VArg{P.vt.p, 4 * DN};
  pa.mixed = mixed ? 1 : 0;
  pa.vt32 = VArg32{P.vt32.p, 4 * DN};
  pa.z32 = VArg32{P.z32.p, P.ld};
  pa.pt = VArg{P.pt.p, npt * m->nv};
  pa.vmg = vmg ? 1 : 0;
  pa.pmg = pmg ? 1 : 0;
  pa.mg_nu = o->mg_smooth;
  pa.mg_post0 = o->mg_post0;
  pa.mg_ratio = o->mg_ratio;
  if (vmg || pmg)
    mg_assign(m, B, esz, vmg, pmg, P.mgbuf.p, mixed ? (void*)P.vt32.p : (void*)P.vt.p, (void*)P.pt.p, P.mglam.p,
              pa.mg);
  pa.mg.vinv = mixed ? (const void*)P.mginv32.p : (const void*)P.mginv.p;
  std::vector<int> all(B);
  for (int k = 0; k < B; ++k) all[k] = k;
  SCVS_HIP(hipMemcpyAsync(P.act_all.p, all.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
  P.act_new.alloc(B);
  int rc = SCVS_OK;
  // Work queue over the slots: a slot whose system has finished takes the next pending
  // system at the next restart boundary, so a batch never waits for its slowest system
  // with idle slots. Largest work first: steady systems (w = 0) take the most
  // iterations and start first; the others keep their order.
  std::vector<int64_t> queue;
  for (int64_t k = 0; k < nsys; ++k)
    if (omega[k] == 0.0) queue.push_back(k);
  for (int64_t k = 0; k < nsys; ++k)
    if (omega[k] != 0.0) queue.push_back(k);
  size_t qnext = 0;
  std::vector<int64_t> sys_of(B, -1);  // system held by each slot (-1: free)
  std::vector<int> iters(B, 0), cycles(B, 0), warm(B, 0);
  std::vector<double> info(4 * B);
  Batch b;
  b.nact = B;
  b.act = P.act_all;
  b.omega = P.omega;
  b.lv = P.lv;
  b.pen = o->penalty / m->mu;
  b.wsteady = o->steady_schur_omega;
  const double2* gp = (const double2*)g;
  const double2* x0p = (const double2*)x0;
  // initial residual into V_0 of every listed slot, and its norm
  auto residual0 = [&](const Batch& bb, const KArgs& ka, dim3 gn) {
    const int64_t vst = (int64_t)(mk + 1) * P.ld;
    if (P.v32) {
      spmv_resid32(m, bb, P.X(), VArg32{reinterpret_cast<float2*>(P.V.p), vst}, P.F(), s, P.T());
      k_norm<1, float2><<<gn, RBS, 0, s>>>(ka, VArg{}, o->rtol, o->inner_rtol);
    } else {
      spmv_full(m, bb, P.X(), VArg{P.V.p, vst}, SPMV_RESID, true, P.F(), nullptr, s);
      k_norm<1, double2><<<gn, RBS, 0, s>>>(ka, VArg{}, o->rtol, mixed ? o->inner_rtol : 0.0);
    }
  };
  // the initial guess (x0, else zero) with the system's Dirichlet data in the listed slots
  auto init_x = [&](const std::vector<int>& slots, bool use_x0) {
    for (size_t i = 0; i < slots.size(); ++i) {
      const int k = slots[i];
      const int first = (int)(sys_of[k] - k);  // k_init_x reads system first + slot
      const dim3 g1(256, 1);
      const int* ak = P.act_all.p + k;
      if (D == 2)
        k_init_x<2><<<g1, 256, 0, s>>>(P.X(), use_x0 ? x0p : nullptr, use_x0 ? ndof : 0, gp, m->ndir * D, m->dmask,
                                       m->dirnodes, m->ndir, m->n2, ndof, ak, first);
      else
        k_init_x<3><<<g1, 256, 0, s>>>(P.X(), use_x0 ? x0p : nullptr, use_x0 ? ndof : 0, gp, m->ndir * D, m->dmask,
                                       m->dirnodes, m->ndir, m->n2, ndof, ak, first);
    }
    launch_check(s);
  };
  // loads the systems of sys_of into the listed slots: solver state, right-hand side and
  // its norm, preconditioner bounds, initial guess and residual
  auto load = [&](const std::vector<int>& slots) {
    const int n = (int)slots.size();
    for (int k : slots) {
      const int64_t sy = sys_of[k];
      SCVS_HIP(hipMemcpyAsync(P.omega.p + k, omega + sy, sizeof(double), hipMemcpyHostToDevice, s));
      if (ntr)
        SCVS_HIP(hipMemcpyAsync(P.trac.p + (int64_t)k * ntr, traction + 2 * sy * ntr, sizeof(double2) * ntr,
                                hipMemcpyHostToDevice, s));
      iters[k] = cycles[k] = 0;
      warm[k] = x0 ? 1 : 0;
    }
    SCVS_HIP(hipMemcpyAsync(P.act_new.p, slots.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    Batch bs = b;
    bs.nact = n;
    bs.act = P.act_new;
    k_zero_at<<<(n + 63) / 64, 64, 0, s>>>(P.lv, P.act_new, n);
    k_init_state<<<(n + 63) / 64, 64, 0, s>>>(P.st, P.act_new, n);
    // right-hand sides: F = RHS(x_g) with T holding the Dirichlet lift
    for (int k : slots) {
      const int first = (int)(sys_of[k] - k);
      const int* ak = P.act_all.p + k;
      if (D == 2)
        k_init_x<2><<<dim3(256, 1), 256, 0, s>>>(P.T(), nullptr, 0, gp, m->ndir * D, m->dmask, m->dirnodes, m->ndir,
                                                 m->n2, ndof, ak, first);
      else
        k_init_x<3><<<dim3(256, 1), 256, 0, s>>>(P.T(), nullptr, 0, gp, m->ndir * D, m->dmask, m->dirnodes, m->ndir,
                                                 m->n2, ndof, ak, first);
    }
    init_x(slots, x0 != nullptr);
    spmv_full(m, bs, P.T(), P.F(), SPMV_RHS, false, VArg{}, P.trac, s);
    const int nchn = choose_nch(n, ndof);
    KArgs an = kargs(P, ndof, nchn);
    an.act = P.act_new;
    const dim3 gn((unsigned)nchn, (unsigned)n);
    k_norm<0><<<gn, RBS, 0, s>>>(an, P.F(), o->rtol);
    if (vmg)
      mg_prepare(m, bs, P.mglam.p, B, P.mginv.p, mixed ? P.mginv32.p : nullptr, s);
    else
      velocity_bounds(m, bs, P.lv, s);
    residual0(bs, an, gn);
    launch_check(s);
    if (x0) {
      // keep a supplied initial guess only where its residual is below ||f||
      download(info.data(), P.info.p, 4 * B, s);
      std::vector<int> back;
      for (int k : slots)
        if (!(info[4 * k] < 1.0)) {
          back.push_back(k);
          warm[k] = 0;
        }
      if (!back.empty()) {
        SCVS_HIP(hipMemcpyAsync(P.act_new.p, back.data(), sizeof(int) * back.size(), hipMemcpyHostToDevice, s));
        Batch bb = b;
        bb.nact = (int)back.size();
        bb.act = P.act_new;
        KArgs ab = kargs(P, ndof, choose_nch(bb.nact, ndof));
        ab.act = P.act_new;
        init_x(back, false);
        residual0(bb, ab, dim3((unsigned)ab.nch, (unsigned)bb.nact));
        launch_check(s);
      }
    }
  };
  // a finished slot: its solution to the outputs and its report
  auto finish = [&](int k) {
    const int64_t sy = sys_of[k];
    k_copy_out<<<dim3(256, 1), 256, 0, s>>>(P.X(), P.act_all.p + k, (int)sy, 1, m->n2, D, m->nv, (double2*)u_out,
                                            (double2*)p_out);
    launch_check(s);
    if (rep) {
      scvs_report& r = rep[sy];
      const double rel = info[4 * k];
      r.iterations = iters[k];
      r.restarts = cycles[k];
      r.rel_residual = rel;
      r.status = (info[4 * k + 2] != 0.0 || !std::isfinite(rel)) ? 3 : (rel <= o->rtol ? 0 : 1);
      r.warm = warm[k];
    }
    sys_of[k] = -1;
  };
  {
    std::vector<int> fill;
    for (int k = 0; k < B && qnext < queue.size(); ++k) {
      sys_of[k] = queue[qnext++];
      fill.push_back(k);
    }
    load(fill);
  }
  // captured graphs keyed by (kind: 0 steps of all active systems, 1 steps of the
  // still-running subset, 2 cycle end; systems in the launch; chunk index)
  std::map<std::tuple<int, int, int>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  const int chunk = std::min(mk, 30);
  std::vector<int> act_prev;
  for (;;) {
    download(info.data(), P.info.p, 4 * B, s);
    m->ctx->prof.resolve();
    std::vector<int> act, freed;
    for (int k = 0; k < B; ++k) {
      if (sys_of[k] < 0) continue;
      const double rel = info[4 * k];
      if (rel <= o->rtol || info[4 * k + 2] != 0.0 || !std::isfinite(rel) || iters[k] >= o->max_iters) {
        finish(k);
        freed.push_back(k);
        continue;
      }
      act.push_back(k);
    }
    if (o->verbose) {
      fprintf(stderr, "[scvs] slots %d active %zu pending %zu:", B, act.size(), queue.size() - qnext);
      for (int k = 0; k < B && k < 24; ++k) fprintf(stderr, " %.2e", sys_of[k] >= 0 ? info[4 * k] : 0.0);
      fprintf(stderr, "\n");
    }
    if (!freed.empty() && qnext < queue.size()) {
      std::vector<int> fill;
      for (int k : freed)
        if (qnext < queue.size()) {
          sys_of[k] = queue[qnext++];
          fill.push_back(k);
        }
      load(fill);
      continue;  // the new systems' initial residuals decide whether they run
    }
    if (act.empty()) break;
    if (act != act_prev) {
      SCVS_HIP(hipMemcpyAsync(P.act.p, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, s));
      act_prev = act;
    }
    Batch bc = b;
    bc.nact = (int)act.size();
    bc.act = P.act;
    const int na = bc.nact;
    // the cycle runs in chunks of steps; between chunks the host drops the systems that
    // stopped, and the cycle ends as soon as none is running
    const bool use_graph = o->use_graph && !m->ctx->prof.on;
    auto launch = [&](std::tuple<int, int, int> key, const std::function<void(hipStream_t)>& body) {
      if (!use_graph) {
        body(s);
        return;
      }
      auto it = graphs.find(key);
      if (it == graphs.end()) {
        hipGraph_t gph;
        hipGraphExec_t ex;
        hipStream_t cs = m->ctx->capture;
        SCVS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
          body(cs);
        } catch (...) {
          hipGraph_t bad = nullptr;
          (void)hipStreamEndCapture(cs, &bad);
          if (bad) (void)hipGraphDestroy(bad);
          (void)hipGetLastError();
          throw;
        }
        SCVS_HIP(hipStreamEndCapture(cs, &gph));
        SCVS_HIP(hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0));
        it = graphs.emplace(key, std::make_pair(gph, ex)).first;
      }
      SCVS_HIP(hipGraphLaunch(it->second.second, s));
      SCVS_HIP(hipGetLastError());
    };
    std::vector<int> run = act;
    std::vector<int> stops(na), jend(B, mk);
    for (int j0 = 0; j0 < mk; j0 += chunk) {
      const int j1 = std::min(mk, j0 + chunk);
      const bool all_run = run.size() == act.size();
      Batch br = bc;
      br.nact = (int)run.size();
      br.act = all_run ? P.act.p : P.act_run.p;
      launch(std::make_tuple(all_run ? 0 : 1, br.nact, j0 / chunk),
             [&](hipStream_t st) { cycle_steps(m, P, br, pa, ndof, j0, j1, lagged, st); });
      const bool prof_on = m->ctx->prof.on;
      if (j1 == mk && !prof_on) break;
      k_stops<<<(br.nact + 63) / 64, 64, 0, s>>>(P.st, br.act, br.nact, P.stops);
      launch_check(s);
      download(stops.data(), P.stops.p, br.nact, s);
      std::vector<int> next;
      for (int k = 0; k < br.nact; ++k) {
        const int J = stops[k];
        if (J < 0) {
          next.push_back(run[k]);
          continue;
        }
        jend[run[k]] = J;
        // Arnoldi launches of steps J.. returned at once (lagged: pass 2 from J, pass 1 from
        // J + 1, since pass 1 of step J found the stop): take back their bytes
        for (int jj = std::max(J, j0); jj < j1; ++jj) {
          const double v = (double)ndof * (P.v32 ? 8.0 : 16.0);
          if (lagged) {
            if (jj > J) m->ctx->prof.correct("k_lag_dots", -v * (jj + 2));
            m->ctx->prof.correct("k_lag_update", -v * (jj + 4));
          } else {
            m->ctx->prof.correct("k_dots1", -v * (jj + 2));
            m->ctx->prof.correct("k_upd_dots", -v * (jj + 3));
            m->ctx->prof.correct("k_update2", -v * (jj + 3));
          }
        }
      }
      if (next.empty() || j1 == mk) break;
      if (next.size() != run.size()) {
        SCVS_HIP(hipMemcpyAsync(P.act_run.p, next.data(), sizeof(int) * next.size(), hipMemcpyHostToDevice, s));
        run.swap(next);
      }
    }
    for (int k : act) {
      const double vb = (double)ndof * (P.v32 ? 8.0 : 16.0);
      m->ctx->prof.correct("k_combine", -vb * (mk - jend[k]));
      if (lagged && jend[k] < mk) m->ctx->prof.correct("k_lag_dots", -vb * (mk + 1));
    }
    launch(std::make_tuple(2, na, 0),
           [&](hipStream_t st) { cycle_end(m, P, bc, pa, ndof, o->rtol, o->inner_rtol, lagged, st); });
    // this cycle's iterations (the cycle end wrote them beside the new residuals)
    download(info.data(), P.info.p, 4 * B, s);
    for (int k : act) {
      iters[k] += (int)info[4 * k + 1];
      cycles[k]++;
    }
  }
  for (auto& kv : graphs) {
    (void)hipGraphExecDestroy(kv.second.second);
    (void)hipGraphDestroy(kv.second.first);
  }
  SCVS_HIP(hipStreamSynchronize(s));
  return rc;
}

}  // namespace scvs

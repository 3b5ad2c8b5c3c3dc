// Row-group lane maps and Chebyshev recurrence scalars shared by the row kernels
// (operator, preconditioner, multigrid).
//
// A row of a sparse pattern is handled by a group of W lanes (a power of two, so
// shuffles stay inside the group); the group's lanes cover the row's (system,
// component) pairs, G of them, in passes of UL lanes when G exceeds one group.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace scvs {

struct LaneMap {
  int G;     // (system, component) pairs per row
  int W;     // lanes per row group (a power of two, <= 64)
  int UL;    // pair lanes used per pass (a multiple of D, <= W)
  int R;     // rows per wavefront (64 / W)
  int iters; // passes over the pairs
};

// Rows are handled by groups of W lanes (a power of two, so shuffles can stay
// inside a group); the group's lanes cover the (system, component) pairs.
inline LaneMap lane_map(int nact, int D) {
  const int G = nact * D;
  if (G <= 32) {
    int W = 1;
    while (W < G) W <<= 1;
    return {G, W, G, 64 / W, 1};
  }
  const int UL = (64 / D) * D;
  return {G, 64, UL, 1, (G + UL - 1) / UL};
}

struct Lane {
  int64_t row;
  int li;     // lane within the row group
  int p0;     // first pair of this lane
  bool rowok;
  bool pairok0;
};

// Workgroups are dealt to the 8 XCDs in turn. Within every group of 8 * XRUN
// consecutive workgroups, XCD x takes the XRUN consecutive row blocks starting at
// x * XRUN, so that neighbouring rows (whose gathers overlap) share one XCD's L2 while
// all XCDs stay in the same stretch of rows; a ragged last group keeps its order.
constexpr int64_t XRUN = 16;
__device__ __forceinline__ int64_t row_block() {
  const int64_t b = blockIdx.x, S = 8 * XRUN, g = b / S;
  if ((g + 1) * S > (int64_t)gridDim.x) return b;
  const int64_t off = b - g * S;
  return g * S + (off % 8) * XRUN + off / 8;
}

__device__ __forceinline__ Lane lane_of(const LaneMap& lm, int64_t nrows) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  Lane L;
  L.li = lane & (lm.W - 1);
  L.p0 = L.li;
  L.row = (row_block() * 4 + wave) * lm.R + lane / lm.W;
  L.rowok = L.row < nrows;
  L.pairok0 = L.li < lm.UL;
  return L;
}

inline unsigned row_blocks(int64_t nrows, const LaneMap& lm) {
  const int64_t per = 4 * (int64_t)lm.R;
  return (unsigned)((nrows + per - 1) / per);
}

// Chebyshev recurrence scalars for step i >= 1 on [lmax/ratio, lmax]:
// rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1}) with sigma = theta/delta =
// (1 + 1/ratio)/(1 - 1/ratio), which does not depend on lmax; returns rho_{i-1}, rho_i.
// (Computed once per step on the host; the kernels form theta and delta from lmax.)
struct ChebStep {
  double rprev, rcur;
};
inline ChebStep cheb_step(double ratio, int i) {
  const double sigma = (1.0 + 1.0 / ratio) / (1.0 - 1.0 / ratio);
  double r = 1.0 / sigma, rp = r;
  for (int k = 1; k <= i; ++k) {
    rp = r;
    r = 1.0 / (2.0 * sigma - r);
  }
  return {rp, r};
}

}  // namespace scvs

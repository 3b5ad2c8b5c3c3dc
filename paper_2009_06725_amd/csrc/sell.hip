// Sliced rows (layout described with struct Sell): the S2 operator of a mesh (the
// momentum block mu Ks + j w rho M of Eq. linear_sys_def, with the coupling G on the
// vertex-column prefix of each row and G^T on the vertex rows) and the level-0
// operators of the multigrid blocks, in the form the wide row kernels read.
#include <algorithm>
#include <functional>
#include <thread>

#include "internal.hpp"

namespace scvs {
namespace {

int sell_threads() {
  const unsigned t = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(t, 16u));
}

// Column indices: thread per slot, the entries of its row in order, padding with the
// row's own index (slots without a row: column 0).
__global__ void k_sell_col(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                           const int64_t* __restrict__ off, const int32_t* __restrict__ row, int64_t nslot,
                           int32_t* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  const int64_t sl = q / SELL_C, e0 = off[sl] + q % SELL_C;
  const int len = (int)((off[sl + 1] - off[sl]) / SELL_C);
  const int32_t i = row[q];
  const int64_t j0 = i >= 0 ? ptr[i] : 0, rl = i >= 0 ? ptr[i + 1] - j0 : 0;
  for (int t = 0; t < len; ++t) out[e0 + (int64_t)t * SELL_C] = t < rl ? col[j0 + t] : (i >= 0 ? i : 0);
}

// Values from CSR values `a` of the same pattern (zero on padding). With NC > 1 the
// CSR holds NC component arrays of `cst` values each and an entry keeps its NC
// values together: out[e * NC + c] = a[c * cst + j]. `ptr` gives each row's first
// CSR value, `lens` (null: from ptr) its length, `off` the slices' entries.
template <class R, int NC>
__global__ void k_sell_val(const int64_t* __restrict__ ptr, const int32_t* __restrict__ lens,
                           const R* __restrict__ a, int64_t cst, const int64_t* __restrict__ off,
                           const int32_t* __restrict__ row, int64_t nslot, R* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nslot) return;
  const int64_t sl = q / SELL_C, e0 = off[sl] + q % SELL_C;
  const int len = (int)((off[sl + 1] - off[sl]) / SELL_C);
  const int32_t i = row[q];
  const int64_t j0 = i >= 0 ? ptr[i] : 0;
  const int64_t rl = i < 0 ? 0 : (lens ? lens[i] : ptr[i + 1] - j0);
  for (int t = 0; t < len; ++t) {
    const int64_t e = e0 + (int64_t)t * SELL_C;
#pragma unroll
    for (int c = 0; c < NC; ++c) out[e * NC + c] = t < rl ? a[c * cst + j0 + t] : (R)0;
  }
}

// Slots of rows [a, b) sorted by length (longest first, ties by index) in windows of
// SELL_WIN rows, written from `first` on; returns the number of slots (a multiple of
// SELL_C: the last slice of the range is padded with -1).
int64_t order_range(const std::vector<int64_t>& ptr, int64_t a, int64_t b, std::vector<int32_t>& row,
                    int64_t first) {
  const int64_t n = b - a, nsl = (n + SELL_C - 1) / SELL_C, nwin = (n + SELL_WIN - 1) / SELL_WIN;
  const int nt = sell_threads();
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int64_t w = t; w < nwin; w += nt) {
        const int64_t w0 = a + w * SELL_WIN, w1 = std::min(b, w0 + SELL_WIN);
        int32_t* r = row.data() + first + (w0 - a);
        for (int64_t i = w0; i < w1; ++i) r[i - w0] = (int32_t)i;
        std::stable_sort(r, r + (w1 - w0),
                         [&](int32_t x, int32_t y) { return ptr[x + 1] - ptr[x] > ptr[y + 1] - ptr[y]; });
      }
    });
  for (auto& x : th) x.join();
  return nsl * SELL_C;
}

// Per slice: the first row's value of `len` (slices are sorted, so it is the largest)
// unless `maxall`, in which case the maximum over the slice's rows; prefix sums of
// SELL_C times that into off.
std::vector<int64_t> slice_offsets(const std::vector<int32_t>& row, const std::function<int64_t(int32_t)>& len,
                                   bool maxall) {
  const int64_t nsl = (int64_t)row.size() / SELL_C;
  std::vector<int64_t> off(nsl + 1, 0);
  for (int64_t sl = 0; sl < nsl; ++sl) {
    int64_t l = 0;
    for (int r = 0; r < (maxall ? SELL_C : 1); ++r) {
      const int32_t i = row[sl * SELL_C + r];
      if (i >= 0) l = std::max(l, len(i));
    }
    off[sl + 1] = off[sl] + l * SELL_C;
  }
  return off;
}

}  // namespace

void sell_build(Sell& S, const std::vector<int64_t>& ptr, int64_t n, int64_t split, const int64_t* dptr,
                const int32_t* dcol, hipStream_t s) {
  const int64_t n0 = (split + SELL_C - 1) / SELL_C * SELL_C, n1 = (n - split + SELL_C - 1) / SELL_C * SELL_C;
  std::vector<int32_t> row(n0 + n1, -1);
  order_range(ptr, 0, split, row, 0);
  order_range(ptr, split, n, row, n0);
  S.nslot = n0 + n1;
  S.split_slots = n0;
  const std::vector<int64_t> off = slice_offsets(row, [&](int32_t i) { return ptr[i + 1] - ptr[i]; }, false);
  S.split_entries = off[n0 / SELL_C];
  S.off.upload(off.data(), off.size(), s);
  S.row.upload(row.data(), row.size(), s);
  S.col.alloc((size_t)off.back());
  k_sell_col<<<(unsigned)((S.nslot + 255) / 256), 256, 0, s>>>(dptr, dcol, S.off, S.row, S.nslot, S.col);
  launch_check(s);
  SCVS_HIP(hipStreamSynchronize(s));  // row and off are host temporaries
}

template <class R>
void sell_values(const Sell& S, const int64_t* dptr, const R* a, DBuf<R>& out, hipStream_t s) {
  out.alloc(S.col.n);
  k_sell_val<R, 1><<<(unsigned)((S.nslot + 255) / 256), 256, 0, s>>>(dptr, nullptr, a, 0, S.off, S.row, S.nslot,
                                                                      out);
  launch_check(s);
}
template void sell_values<float>(const Sell&, const int64_t*, const float*, DBuf<float>&, hipStream_t);
template void sell_values<double>(const Sell&, const int64_t*, const double*, DBuf<double>&, hipStream_t);

void s2sell_setup(scvs_mesh m, bool f32, bool f64, hipStream_t s) {
  Sell& S = m->s2sell;
  const int D = m->dim;
  if (!S.off.p) {
    std::vector<int64_t> rp(m->n2 + 1), p21(m->n2 + 1);
    std::vector<int32_t> nvc(m->n2);
    download(rp.data(), m->rowptr.p, m->n2 + 1, s);
    download(p21.data(), m->rowptr21.p, m->n2 + 1, s);
    download(nvc.data(), m->nvc.p, m->n2, s);
    sell_build(S, rp, m->n2, m->nv, m->rowptr, m->col, s);
    std::vector<int32_t> row(S.nslot);
    download(row.data(), S.row.p, S.nslot, s);
    // G entries: per slice the longest vertex-column prefix of its rows
    const std::vector<int64_t> goff = slice_offsets(row, [&](int32_t i) { return (int64_t)nvc[i]; }, true);
    m->s2_goff.upload(goff.data(), goff.size(), s);
    m->s2_gn = goff.back();
    SCVS_HIP(hipStreamSynchronize(s));
  }
  const unsigned nb = (unsigned)((S.nslot + 255) / 256);
  if (f32 && !S.K32.p) {
    sell_values<float>(S, m->rowptr, m->Ks32, S.K32, s);
    sell_values<float>(S, m->rowptr, m->M32, S.M32, s);
    // G^c on the vertex-column prefix (CSR C21 values, D arrays of nnz21), G^T^c on the
    // vertex rows (D arrays of nnzv over the vertex rows' S2 entries)
    m->s2_G32.alloc((size_t)m->s2_gn * D);
    m->s2_Gt32.alloc((size_t)std::max<int64_t>(1, S.split_entries * D));
    if (D == 2) {
      k_sell_val<float, 2><<<nb, 256, 0, s>>>(m->rowptr21, m->nvc, m->G32, m->nnz21, m->s2_goff, S.row, S.nslot,
                                               m->s2_G32);
      k_sell_val<float, 2><<<nb, 256, 0, s>>>(m->rowptr, nullptr, m->Gt32, m->nnzv, S.off, S.row, S.split_slots,
                                               m->s2_Gt32);
    } else {
      k_sell_val<float, 3><<<nb, 256, 0, s>>>(m->rowptr21, m->nvc, m->G32, m->nnz21, m->s2_goff, S.row, S.nslot,
                                               m->s2_G32);
      k_sell_val<float, 3><<<nb, 256, 0, s>>>(m->rowptr, nullptr, m->Gt32, m->nnzv, S.off, S.row, S.split_slots,
                                               m->s2_Gt32);
    }
    launch_check(s);
  }
  if (f64 && !S.K.p) {
    sell_values<double>(S, m->rowptr, m->Ks, S.K, s);
    sell_values<double>(S, m->rowptr, m->M, S.M, s);
  }
  SCVS_HIP(hipStreamSynchronize(s));
}

void s2sell_release_values(scvs_mesh m) {
  m->s2sell.K32.release();
  m->s2sell.M32.release();
  m->s2sell.K.release();
  m->s2sell.M.release();
  m->s2_G32.release();
  m->s2_Gt32.release();
}

}  // namespace scvs

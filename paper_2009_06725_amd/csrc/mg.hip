// Aggregation multigrid for the two blocks of the preconditioner (section 2.3:
// the velocity block mu Ks + j w rho M of Eq. linear_sys_def, and the pressure
// Laplacian of the Schur approximation mu Mp^-1 + j w rho L^-1).
//
// The paper preconditions GMRES with Jacobi and names better solvers for the
// unstabilized system as the way to cut its iteration counts. Here each block
// gets one V-cycle per application:
//   * velocity: level 0 is the quadratic pattern itself (free nodes; the same
//     scalar operator for every component). Level 1 is the linear space on the
//     same mesh: P2 contains P1, so the nested transfer is exact (a vertex keeps
//     its value, an edge node takes the mean of its two ends; Dirichlet nodes
//     are left out), and its Galerkin products P^T Ks P, P^T M P are the linear
//     stiffness and mass. Below that, smoothed aggregation of the linear
//     stiffness: greedy aggregates of strongly coupled nodes, the piecewise
//     constant transfer smoothed by one damped Jacobi step, and Galerkin
//     products of both matrices. Every level keeps Ks and M apart, so one
//     hierarchy serves every frequency: the level operator of system s is
//     mu K_l + j w_s rho M_l;
//   * pressure: the same aggregation on the assembled Laplacian L (no mass).
// Smoothing is a Chebyshev iteration in D^-1 A with D the complex diagonal of
// the level operator, on [lambda/ratio, lambda], lambda a Gershgorin bound of
// |D^-1 A| per system and level; the coarsest level (at most MG_COARSE_MAX rows)
// is solved with its dense inverse. The hierarchy is built on the host once per
// assembly and boundary-condition set and lives on the device. Level 0 of both
// hierarchies is also kept in sliced rows (Sell), which its smoothing and residual
// kernels read: one lane per (row, system) walks the row with coalesced loads.
//
// Vectors of one level are interleaved [n_l][G]: pair p = (system index in the
// batch) * PD + component (PD = dim for the velocity, 1 for the pressure), so
// one column index gathers the values of every system and component at once.
#include <algorithm>
#include <thread>

#include "internal.hpp"
#include "rowmap.hpp"

namespace scvs {
namespace {

// ---------------- host: sparse matrices and the aggregation hierarchy ----------------
struct HCsr {
  int64_t n = 0, m = 0;  // rows, columns
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> a, b;  // values; b (a second value array) may be empty
  int64_t nnz() const { return ptr.empty() ? 0 : ptr[n]; }
};

int host_threads() {
  const unsigned t = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(t, 16u));
}

// Runs f(r0, r1, t) over nt contiguous row ranges in parallel.
template <class F>
int parallel_rows(int64_t n, F&& f) {
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), n / 2048));
  if (nt == 1) {
    f((int64_t)0, n, 0);
    return 1;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) th.emplace_back([&, t] { f(n * t / nt, n * (t + 1) / nt, t); });
  for (auto& x : th) x.join();
  return nt;
}

// C = A B, rows in parallel (Gustavson with a dense accumulator per thread), columns
// sorted. At most one factor carries a second value array; C then carries
// a = A.a B.a and b = (A.b B.a or A.a B.b).
HCsr spgemm(const HCsr& A, const HCsr& B) {
  const bool twoA = !A.b.empty(), twoB = !B.b.empty();
  const bool two = twoA || twoB;
  struct Part {
    std::vector<int64_t> cnt;
    std::vector<int32_t> col;
    std::vector<double> a, b;
  };
  std::vector<Part> parts(host_threads());
  std::vector<std::pair<int64_t, int64_t>> ranges(host_threads());
  const int nt = parallel_rows(A.n, [&](int64_t r0, int64_t r1, int t) {
    Part& P = parts[t];
    ranges[t] = {r0, r1};
    std::vector<int64_t> mark(B.m, -1);
    std::vector<double> acc_a(B.m, 0.0), acc_b(two ? B.m : 0, 0.0);
    std::vector<int32_t> row;
    for (int64_t i = r0; i < r1; ++i) {
      row.clear();
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
        const int32_t j = A.col[k];
        const double aa = A.a[k], ab = twoA ? A.b[k] : 0.0;
        for (int64_t q = B.ptr[j]; q < B.ptr[j + 1]; ++q) {
          const int32_t c = B.col[q];
          if (mark[c] != i) {
            mark[c] = i;
            acc_a[c] = 0.0;
            if (two) acc_b[c] = 0.0;
            row.push_back(c);
          }
          acc_a[c] += aa * B.a[q];
          if (twoA) acc_b[c] += ab * B.a[q];
          if (twoB) acc_b[c] += aa * B.b[q];
        }
      }
      std::sort(row.begin(), row.end());
      P.cnt.push_back((int64_t)row.size());
      for (int32_t c : row) {
        P.col.push_back(c);
        P.a.push_back(acc_a[c]);
        if (two) P.b.push_back(acc_b[c]);
      }
    }
  });
  HCsr C;
  C.n = A.n;
  C.m = B.m;
  C.ptr.assign(A.n + 1, 0);
  for (int t = 0; t < nt; ++t) {
    const int64_t r0 = ranges[t].first;
    for (size_t k = 0; k < parts[t].cnt.size(); ++k) C.ptr[r0 + (int64_t)k + 1] = parts[t].cnt[k];
  }
  for (int64_t i = 0; i < A.n; ++i) C.ptr[i + 1] += C.ptr[i];
  C.col.resize(C.ptr[A.n]);
  C.a.resize(C.ptr[A.n]);
  if (two) C.b.resize(C.ptr[A.n]);
  parallel_rows(nt, [&](int64_t t0, int64_t t1, int) {
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t off = C.ptr[ranges[t].first];
      std::copy(parts[t].col.begin(), parts[t].col.end(), C.col.begin() + off);
      std::copy(parts[t].a.begin(), parts[t].a.end(), C.a.begin() + off);
      if (two) std::copy(parts[t].b.begin(), parts[t].b.end(), C.b.begin() + off);
    }
  });
  return C;
}

// Transpose of a one-valued matrix; each row of the result has ascending columns.
HCsr transpose(const HCsr& P) {
  HCsr R;
  R.n = P.m;
  R.m = P.n;
  R.ptr.assign(R.n + 1, 0);
  for (int64_t k = 0; k < P.nnz(); ++k) R.ptr[P.col[k] + 1]++;
  for (int64_t i = 0; i < R.n; ++i) R.ptr[i + 1] += R.ptr[i];
  R.col.resize(P.nnz());
  R.a.resize(P.nnz());
  std::vector<int64_t> pos(R.ptr.begin(), R.ptr.end() - 1);
  for (int64_t i = 0; i < P.n; ++i)
    for (int64_t k = P.ptr[i]; k < P.ptr[i + 1]; ++k) {
      const int64_t q = pos[P.col[k]]++;
      R.col[q] = (int32_t)i;
      R.a[q] = P.a[k];
    }
  return R;
}

double diag_of(const HCsr& A, int64_t i) {
  for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
    if (A.col[k] == i) return A.a[k];
  return 0.0;
}

// Greedy aggregation on the strong couplings: a node whose strong neighbours are all
// free starts an aggregate with them; a leftover node joins the aggregate of its first
// aggregated strong neighbour; what is still left starts aggregates with its free
// strong neighbours. Strength: with theta > 0, |a_ij| >= theta sqrt(a_ii a_jj) (the
// first aggregation, on the sparse linear-element operators); with theta < 0,
// |a_ij| >= |theta| max_k |a_ik| over the row's off-diagonals (the deeper, denser
// levels, where every single coupling is small against the diagonal). Returns the
// aggregate of every node and the count.
std::vector<int32_t> aggregate(const HCsr& A, double theta, int32_t& na) {
  const int64_t n = A.n;
  std::vector<double> d(n), mx(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    d[i] = std::fabs(diag_of(A, i));
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] != i) mx[i] = std::max(mx[i], std::fabs(A.a[k]));
  }
  auto strong = [&](int64_t i, int64_t k) {
    const int32_t j = A.col[k];
    if (j == i) return false;
    if (theta < 0.0) return mx[i] > 0.0 && std::fabs(A.a[k]) >= -theta * mx[i];
    return std::fabs(A.a[k]) >= theta * std::sqrt(d[i] * d[j]);
  };
  std::vector<int32_t> agg(n, -1);
  na = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1] && free; ++k)
      if (strong(i, k) && agg[A.col[k]] >= 0) free = false;
    if (!free) continue;
    agg[i] = na;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k)) agg[A.col[k]] = na;
    ++na;
  }
  std::vector<int32_t> first(agg);
  for (int64_t i = 0; i < n; ++i) {
    if (first[i] >= 0) continue;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k) && first[A.col[k]] >= 0) {
        agg[i] = first[A.col[k]];
        break;
      }
  }
  for (int64_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k) && agg[A.col[k]] < 0) agg[A.col[k]] = na;
    ++na;
  }
  return agg;
}

// max_i sum_j |a_ij| / a_ii
double gershgorin(const HCsr& A) {
  double lam = 0.0;
  for (int64_t i = 0; i < A.n; ++i) {
    double s = 0.0, dg = 0.0;
    for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      s += std::fabs(A.a[k]);
      if (A.col[k] == i) dg = A.a[k];
    }
    if (dg > 0.0) lam = std::max(lam, s / dg);
  }
  return lam;
}

// P = (I - w D^-1 A) T with T the aggregate indicator and w = 4 / (3 lambda),
// truncated (below).
HCsr smoothed_prolongator(const HCsr& A, const std::vector<int32_t>& agg, int32_t na) {
  const double w = 4.0 / (3.0 * std::max(gershgorin(A), 1e-300));
  HCsr P;
  P.n = A.n;
  P.m = na;
  P.ptr.assign(A.n + 1, 0);
  std::vector<int64_t> mark(na, -1);
  std::vector<double> acc(na, 0.0);
  std::vector<int32_t> row;
  for (int64_t i = 0; i < A.n; ++i) {
    row.clear();
    const double dg = diag_of(A, i);
    auto add = [&](int32_t c, double v) {
      if (mark[c] != i) {
        mark[c] = i;
        acc[c] = 0.0;
        row.push_back(c);
      }
      acc[c] += v;
    };
    add(agg[i], 1.0);
    if (dg != 0.0)
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k) add(agg[A.col[k]], -w * A.a[k] / dg);
    std::sort(row.begin(), row.end());
    // truncation: entries below 5% of the row's largest are dropped and the rest rescaled
    // to keep the row sum (the coarse operators of wide stencils stay sparse)
    double amax = 0.0, sall = 0.0, skeep = 0.0;
    for (int32_t c : row) amax = std::max(amax, std::fabs(acc[c]));
    for (int32_t c : row) {
      sall += acc[c];
      if (std::fabs(acc[c]) >= 0.05 * amax) skeep += acc[c];
    }
    const double sc = skeep != 0.0 ? sall / skeep : 1.0;
    for (int32_t c : row)
      if (std::fabs(acc[c]) >= 0.05 * amax) {
        P.col.push_back(c);
        P.a.push_back(acc[c] * sc);
      }
    P.ptr[i + 1] = (int64_t)P.col.size();
  }
  return P;
}

// ---------------- host -> device ----------------
template <class T>
void up(DBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  d.upload(h.data(), h.size(), s);
}
void up32(DBuf<float>& d, const std::vector<double>& h, hipStream_t s) {
  std::vector<float> f(h.begin(), h.end());
  d.upload(f.data(), f.size(), s);
  SCVS_HIP(hipStreamSynchronize(s));  // f is a temporary
}

// (every upload helper synchronizes before its host vectors go out of scope)
void upload_level(MgLevel& L, const HCsr& A, hipStream_t s) {
  L.n = A.n;
  L.nnz = A.nnz();
  up(L.ptr, A.ptr, s);
  up(L.col, A.col, s);
  up(L.K, A.a, s);
  up32(L.K32, A.a, s);
  std::vector<double> kd(A.n), md(A.n, 0.0);
  for (int64_t i = 0; i < A.n; ++i) kd[i] = diag_of(A, i);
  if (!A.b.empty()) {
    up(L.M, A.b, s);
    up32(L.M32, A.b, s);
    for (int64_t i = 0; i < A.n; ++i)
      for (int64_t k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        if (A.col[k] == i) md[i] = A.b[k];
  }
  up(L.Kd, kd, s);
  up32(L.Kd32, kd, s);
  up(L.Md, md, s);
  up32(L.Md32, md, s);
  L.lam = gershgorin(A);
  SCVS_HIP(hipStreamSynchronize(s));
}

void upload_transfer(MgLevel& L, const HCsr& P, hipStream_t s) {
  const HCsr R = transpose(P);
  L.nc = P.m;
  up(L.pptr, P.ptr, s);
  up(L.pcol, P.col, s);
  up(L.pval, P.a, s);
  up32(L.pval32, P.a, s);
  up(L.rptr, R.ptr, s);
  up(L.rcol, R.col, s);
  up(L.rval, R.a, s);
  up32(L.rval32, R.a, s);
  SCVS_HIP(hipStreamSynchronize(s));
}

// Aggregation levels from A down: appends levels and the transfers between them until a
// level has at most `coarse_max` rows (it is then inverted densely). The first
// aggregation uses symmetric strength theta, the deeper ones row-relative strength 0.25
// (0.1 when that leaves the level nearly uncoarsened).
void build_below(MgHier& H, HCsr A, int coarse_max, double theta, hipStream_t s) {
  const size_t first_level = H.lv.size();
  for (;;) {
    H.lv.emplace_back();
    MgLevel& L = H.lv.back();
    if (A.n <= coarse_max) {
      upload_level(L, A, s);
      break;
    }
    SCVS_REQUIRE(H.lv.size() < (size_t)MG_MAXLEV, SCVS_E_CAPACITY, "multigrid hierarchy too deep");
    int32_t na = 0;
    // first aggregation of this hierarchy: symmetric strength; deeper: row-relative
    const bool first = H.lv.size() == first_level + 1;
    std::vector<int32_t> agg = aggregate(A, first ? theta : -0.25, na);
    if (na >= A.n * 0.85) agg = aggregate(A, -0.1, na);  // more couplings count as strong
    SCVS_REQUIRE(na < A.n * 0.85 && na >= 1, SCVS_E_CAPACITY, "multigrid coarsening stalled");
    const HCsr P = smoothed_prolongator(A, agg, na);
    HCsr AP = spgemm(A, P);
    HCsr Ac = spgemm(transpose(P), AP);
    upload_level(L, A, s);
    upload_transfer(L, P, s);
    if (H.lv.size() > 1 && A.n >= MG_SELL_MIN) {  // large coarse levels: sliced rows too
      sell_build(L.sell, A.ptr, A.n, A.n, L.ptr, L.col, s);
      sell_values<double>(L.sell, L.ptr, L.K.p, L.sell.K, s);
      sell_values<float>(L.sell, L.ptr, L.K32.p, L.sell.K32, s);
      if (!A.b.empty()) {
        sell_values<double>(L.sell, L.ptr, L.M.p, L.sell.M, s);
        sell_values<float>(L.sell, L.ptr, L.M32.p, L.sell.M32, s);
      }
      SCVS_HIP(hipStreamSynchronize(s));
    }
    A = std::move(Ac);
  }
}

// In-place inverse of a dense n x n matrix by Gauss-Jordan elimination without
// pivoting (the coarse operators have a symmetric positive definite real part, so
// every leading block is nonsingular). A zero pivot belongs to a row and column
// without couplings; they stay zero (that unknown is left out).
void dense_inverse(std::vector<double>& a, int64_t n) {
  std::vector<double> rk(n);
  for (int64_t k = 0; k < n; ++k) {
    if (a[k * n + k] == 0.0) continue;
    const double pinv = 1.0 / a[k * n + k];
    for (int64_t j = 0; j < n; ++j) rk[j] = (j == k ? 1.0 : a[k * n + j]) * pinv;
    for (int64_t i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[i * n + k];
      for (int64_t j = 0; j < n; ++j) a[i * n + j] = (j == k ? 0.0 : a[i * n + j]) - f * rk[j];
    }
    for (int64_t j = 0; j < n; ++j) a[k * n + j] = rk[j];
  }
}

}  // namespace

// Builds both hierarchies of a mesh (after assembly and boundary conditions).
void mg_setup(scvs_mesh m, hipStream_t s) {
  if (m->mg && m->mg->gen == m->generation) return;
  auto mg = std::make_unique<MgData>();
  mg->gen = m->generation;
  const int64_t n2 = m->n2, nv = m->nv, nnz = m->nnz, ne = m->ne;
  // host copies of the quadratic pattern, Ks, M, the Dirichlet mask and the edges
  std::vector<int64_t> rp(n2 + 1);
  std::vector<int32_t> col(nnz), dm(n2), ed(2 * ne);
  std::vector<double> ks(nnz), mm(nnz);
  download(rp.data(), m->rowptr.p, n2 + 1, s);
  download(col.data(), m->col.p, nnz, s);
  download(ks.data(), m->Ks.p, nnz, s);
  download(mm.data(), m->M.p, nnz, s);
  download(dm.data(), m->dmask.p, n2, s);
  download(ed.data(), m->edges.p, 2 * ne, s);
  // nested transfer P2 -> P1 on free nodes: coarse unknowns are the free vertices
  std::vector<int32_t> cidx(nv, -1);
  int32_t nc = 0;
  for (int64_t v = 0; v < nv; ++v)
    if (dm[v] == 0) cidx[v] = nc++;
  HCsr P0;
  P0.n = n2;
  P0.m = nc;
  P0.ptr.assign(n2 + 1, 0);
  for (int64_t A = 0; A < n2; ++A) {
    if (dm[A] == 0) {
      if (A < nv) {
        P0.col.push_back(cidx[A]);
        P0.a.push_back(1.0);
      } else {
        int32_t a = ed[2 * (A - nv)], b = ed[2 * (A - nv) + 1];
        if (a > b) std::swap(a, b);
        for (int32_t v : {a, b})
          if (cidx[v] >= 0) {
            P0.col.push_back(cidx[v]);
            P0.a.push_back(0.5);
          }
      }
    }
    P0.ptr[A + 1] = (int64_t)P0.col.size();
  }
  // level-1 operators P0^T [Ks, M] P0 (Dirichlet rows of P0 are empty, so the
  // Dirichlet rows and columns of Ks and M drop out)
  HCsr A0;
  A0.n = A0.m = n2;
  A0.ptr = std::move(rp);
  A0.col = std::move(col);
  A0.a = std::move(ks);
  A0.b = std::move(mm);
  HCsr A1 = spgemm(transpose(P0), spgemm(A0, P0));
  A0 = HCsr();
  MgHier& V = mg->vel;
  V.lv.emplace_back();
  V.lv[0].n = n2;
  V.lv[0].nnz = nnz;
  upload_transfer(V.lv[0], P0, s);
  build_below(V, std::move(A1), MG_COARSE_MAX, 0.08, s);
  V.mass = true;
  // pressure: the assembled Laplacian and the levels below it
  HCsr L;
  L.n = L.m = nv;
  L.ptr.resize(nv + 1);
  L.col.resize(m->nnzl);
  L.a.resize(m->nnzl);
  download(L.ptr.data(), m->lp_ptr.p, nv + 1, s);
  download(L.col.data(), m->lp_col.p, m->nnzl, s);
  download(L.a.data(), m->lp_val.p, m->nnzl, s);
  sell_build(mg->pres.sell0, L.ptr, nv, nv, m->lp_ptr.p, m->lp_col.p, s);
  build_below(mg->pres, std::move(L), MG_COARSE_MAX, 0.08, s);
  mg->pres.mass = false;
  {
    // the Laplacian's coarsest level is the same for every system: invert it here
    const MgLevel& Lc = mg->pres.lv.back();
    const int64_t n = Lc.n;
    std::vector<int64_t> cp(n + 1);
    std::vector<int32_t> cc(Lc.nnz);
    std::vector<double> cv(Lc.nnz), dn((size_t)n * n, 0.0);
    download(cp.data(), Lc.ptr.p, n + 1, s);
    download(cc.data(), Lc.col.p, Lc.nnz, s);
    download(cv.data(), Lc.K.p, Lc.nnz, s);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = cp[i]; k < cp[i + 1]; ++k) dn[i * n + cc[k]] += cv[k];
    dense_inverse(dn, n);
    std::vector<double2> c2((size_t)n * n);
    std::vector<float2> c32((size_t)n * n);
    for (size_t q = 0; q < c2.size(); ++q) {
      c2[q] = make_double2(dn[q], 0.0);
      c32[q] = make_float2((float)dn[q], 0.0f);
    }
    mg->pres.cinv.upload(c2.data(), c2.size(), s);
    mg->pres.cinv32.upload(c32.data(), c32.size(), s);
  }
  SCVS_HIP(hipStreamSynchronize(s));
  m->mg = std::move(mg);
}

namespace {

// ---------------- device kernels ----------------
template <class R>
struct CplxOf;
template <>
struct CplxOf<double> {
  using C = double2;
};
template <>
struct CplxOf<float> {
  using C = float2;
};

template <class R>
struct LevelArgs {
  int64_t n;
  const int64_t* ptr;
  const int32_t* col;
  const R *K, *M, *Kd, *Md;  // M, Md null: no mass term
  const int32_t* dmask;      // level 0 of the velocity: Dirichlet rows stay zero
  R mu, rho;
};
template <class R>
struct XferArgs {
  int64_t n;
  const int64_t* ptr;
  const int32_t* col;
  const R* v;
};

template <class C>
__device__ __forceinline__ C zero2() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

// a / b for complex a, b; zero for b = 0 (a row without couplings, e.g. a pressure
// vertex whose velocity neighbours are all prescribed, stays zero)
template <class R, class C>
__device__ __forceinline__ C cdiv(C a, R br, R bi) {
  const R den = br * br + bi * bi;
  C r;
  if (den == (R)0) {
    r.x = 0;
    r.y = 0;
    return r;
  }
  r.x = (a.x * br + a.y * bi) / den;
  r.y = (a.y * br - a.x * bi) / den;
  return r;
}

// Per system and level: the Gershgorin bound max_i sum_j |a_ij| / |a_ii| of the level
// operator mu K + j w rho M (FP64 values, free rows and columns). Lanes of a row group
// are the batch's systems; maxima of positive doubles compare as their bit patterns.
template <bool MASS>
__global__ void __launch_bounds__(256) k_mg_bound(LevelArgs<double> la, Batch b, LaneMap lm,
                                                  unsigned long long* __restrict__ out) {
  const Lane L = lane_of(lm, la.n);
  if (!L.rowok) return;
  const int64_t i = L.row;
  if (la.dmask && la.dmask[i] != 0) return;
  for (int it = 0; it < lm.iters; ++it) {
    const int si = L.li + it * lm.UL;
    if (!(L.pairok0 && si < lm.G)) continue;
    const int slot = b.act[si];
    const double wr = MASS ? b.omega[slot] * la.rho : 0.0;
    double s = 0.0;
    for (int64_t k = la.ptr[i]; k < la.ptr[i + 1]; ++k) {
      const int32_t j = la.col[k];
      if (la.dmask && la.dmask[j] != 0) continue;
      const double re = la.mu * la.K[k], im = MASS ? wr * la.M[k] : 0.0;
      s += sqrt(re * re + im * im);
    }
    const double dr = la.mu * la.Kd[i], di = MASS ? wr * la.Md[i] : 0.0;
    const double v = s / sqrt(dr * dr + di * di);
    atomicMax(&out[slot], (unsigned long long)__double_as_longlong(v));
  }
}

// q = sum_j (mu K_ij + j w rho M_ij) x[j] for the lane's pair: the W lanes of a row group
// load W slots of (col, K, M) together and broadcast them by shuffles.
template <class R, bool MASS>
__device__ __forceinline__ typename CplxOf<R>::C level_row(const LevelArgs<R>& la, int W, int li, int64_t i,
                                                           const typename CplxOf<R>::C* __restrict__ x, int G,
                                                           int p, bool ok, R wr) {
  using C = typename CplxOf<R>::C;
  constexpr int U = 8;
  C q = zero2<C>();
  const int64_t j0 = la.ptr[i], j1 = la.ptr[i + 1];
  for (int64_t jb = j0; jb < j1; jb += W) {
    const int n = (int)min((int64_t)W, j1 - jb);
    int32_t mc = 0;
    R mk = 0, mm = 0;
    if (li < n) {
      mc = la.col[jb + li];
      mk = la.K[jb + li];
      if (MASS) mm = la.M[jb + li];
    }
    for (int t = 0; t < n; t += U) {
      int32_t B[U];
      R k[U], m[U];
      C xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = t + u < n ? t + u : 0;
        B[u] = __shfl(mc, src, W);
        k[u] = __shfl(mk, src, W);
        m[u] = MASS ? __shfl(mm, src, W) : (R)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = (ok && t + u < n) ? x[(int64_t)B[u] * G + p] : zero2<C>();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const R kr = la.mu * k[u], ki = wr * m[u];
        q.x += kr * xv[u].x - ki * xv[u].y;
        q.y += kr * xv[u].y + ki * xv[u].x;
      }
    }
  }
  return q;
}

enum { MG_STEP = 0, MG_RESID = 1 };

// One Chebyshev smoothing step on a level (MODE MG_STEP):
//   xn = xk + a (xk - xo) + c D^-1 (bb - A xk),
// first step (first = 1): a = 0, c = 1/theta; later steps: a = rho_k rho_{k-1},
// c = 2 rho_k / delta, with theta, delta from the lane's system bound lambda (xo null: 0).
// MODE MG_RESID: xn = bb - A xk. Lanes cover (row, pair); Dirichlet rows give zero.
template <class R, int PD, bool MASS, int MODE>
__global__ void __launch_bounds__(256) k_mg_step(LevelArgs<R> la, Batch b, LaneMap lm, const double* __restrict__ lam,
                                                 double lamc, double ratio, ChebStep cs, int first,
                                                 const typename CplxOf<R>::C* __restrict__ xk,
                                                 const typename CplxOf<R>::C* __restrict__ xo,
                                                 const typename CplxOf<R>::C* __restrict__ bb,
                                                 typename CplxOf<R>::C* __restrict__ xn) {
  using C = typename CplxOf<R>::C;
  const Lane L = lane_of(lm, la.n);
  if (!L.rowok) return;  // uniform over the row group
  const int64_t i = L.row;
  const bool dir = la.dmask && la.dmask[i] != 0;
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    const bool ok = L.pairok0 && p < lm.G;
    const int si = ok ? p / PD : 0;
    const int slot = b.act[si];
    const R wr = MASS ? (R)(b.omega[slot] * (double)la.rho) : (R)0;
    if (dir) {
      if (ok) xn[i * lm.G + p] = zero2<C>();
      continue;
    }
    const C q = level_row<R, MASS>(la, lm.W, L.li, i, xk, lm.G, p, ok, wr);
    if (!ok) continue;
    const int64_t ki = i * lm.G + p;
    C r = bb[ki];
    r.x -= q.x;
    r.y -= q.y;
    if (MODE == MG_RESID) {
      xn[ki] = r;
      continue;
    }
    const double lm_ = lam ? lam[slot] : lamc;
    const R dr = la.mu * la.Kd[i], di = MASS ? wr * la.Md[i] : (R)0;
    const C d = cdiv<R, C>(r, dr, di);
    R a, c;
    if (first) {
      a = 0;
      c = (R)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)));
    } else {
      a = (R)(cs.rcur * cs.rprev);
      c = (R)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
    }
    const C xv = xk[ki];
    const C xv0 = (xo && !first) ? xo[ki] : zero2<C>();
    C o;
    o.x = xv.x + a * (xv.x - xv0.x) + c * d.x;
    o.y = xv.y + a * (xv.y - xv0.y) + c * d.y;
    xn[ki] = o;
  }
}

// Restriction with the first smoothing step of the coarse level fused in:
// bc[I] = sum_j R_Ij r[j], xc[I] = D_I^-1 bc[I] / theta (coarse bound lambda).
template <class R, int PD, bool MASS>
__global__ void __launch_bounds__(256) k_mg_restrict(XferArgs<R> rt, LevelArgs<R> lc, Batch b, LaneMap lm,
                                                     const double* __restrict__ lam, double lamc, double ratio,
                                                     const typename CplxOf<R>::C* __restrict__ r,
                                                     typename CplxOf<R>::C* __restrict__ bc,
                                                     typename CplxOf<R>::C* __restrict__ xc) {
  using C = typename CplxOf<R>::C;
  const Lane L = lane_of(lm, rt.n);
  if (!L.rowok) return;
  const int64_t I = L.row;
  const int64_t j0 = rt.ptr[I], j1 = rt.ptr[I + 1];
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    const bool ok = L.pairok0 && p < lm.G;
    C acc = zero2<C>();
    for (int64_t jb = j0; jb < j1; jb += lm.W) {
      const int n = (int)min((int64_t)lm.W, j1 - jb);
      int32_t mc = 0;
      R mv = 0;
      if (L.li < n) {
        mc = rt.col[jb + L.li];
        mv = rt.v[jb + L.li];
      }
      for (int t = 0; t < n; ++t) {
        const int32_t j = __shfl(mc, t, lm.W);
        const R w = __shfl(mv, t, lm.W);
        if (ok) {
          const C v = r[(int64_t)j * lm.G + p];
          acc.x += w * v.x;
          acc.y += w * v.y;
        }
      }
    }
    if (!ok) continue;
    const int slot = b.act[p / PD];
    const R wr = MASS ? (R)(b.omega[slot] * (double)lc.rho) : (R)0;
    const double lm_ = lam ? lam[slot] : lamc;
    const R dr = lc.mu * lc.Kd[I], di = MASS ? wr * lc.Md[I] : (R)0;
    const C d = cdiv<R, C>(acc, dr, di);
    const R c = (R)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)));
    const int64_t ki = I * lm.G + p;
    bc[ki] = acc;
    C o;
    o.x = c * d.x;
    o.y = c * d.y;
    xc[ki] = o;
  }
}

// Prolongation and correction: x[i] += sum_J P_iJ e[J].
template <class R>
__global__ void __launch_bounds__(256) k_mg_prolong(XferArgs<R> pt, LaneMap lm,
                                                    const typename CplxOf<R>::C* __restrict__ e,
                                                    typename CplxOf<R>::C* __restrict__ x) {
  using C = typename CplxOf<R>::C;
  const Lane L = lane_of(lm, pt.n);
  if (!L.rowok) return;
  const int64_t i = L.row;
  const int64_t j0 = pt.ptr[i], j1 = pt.ptr[i + 1];
  for (int it = 0; it < lm.iters; ++it) {
    const int p = L.li + it * lm.UL;
    if (!(L.pairok0 && p < lm.G)) continue;
    C acc = zero2<C>();
    for (int64_t k = j0; k < j1; ++k) {
      const C v = e[(int64_t)pt.col[k] * lm.G + p];
      acc.x += pt.v[k] * v.x;
      acc.y += pt.v[k] * v.y;
    }
    const int64_t ki = i * lm.G + p;
    C o = x[ki];
    o.x += acc.x;
    o.y += acc.y;
    x[ki] = o;
  }
}

// ---- long rows (dense coarse levels): S slices of W lanes per row ----
// A block of 256 threads holds RB = 256 / (S W) rows; slice s of a row takes the row's
// chunks of W entries s, s + S, s + 2S, ... and the slices' partial sums meet in LDS,
// where slice 0 adds them in slice order. Short rows keep one W-lane group per row.
struct SplitMap {
  int W, S, RB, UL, G, iters;
};
inline SplitMap split_map(const LaneMap& lm, double avg_row) {
  int S = 1;
  while (2 * S * lm.W <= 256 && 2.0 * S * lm.W <= avg_row) S *= 2;
  return {lm.W, S, 256 / (S * lm.W), lm.UL, lm.G, lm.iters};
}

// sum over slots [j0, j1) of row chunks s, s+S, ... of (ar_j + j ai_j) x[col_j][p] with
// ar = mu K (or the transfer weight), ai = wr M (MASS); every lane of the W-group calls it.
template <class R, bool MASS>
__device__ __forceinline__ typename CplxOf<R>::C slice_row(const int32_t* __restrict__ colv,
                                                           const R* __restrict__ K, const R* __restrict__ Mv,
                                                           R mu, R wr, int W, int S, int s, int li, int64_t j0,
                                                           int64_t j1, const typename CplxOf<R>::C* __restrict__ x,
                                                           int G, int p, bool ok) {
  using C = typename CplxOf<R>::C;
  constexpr int U = 8;
  C q = zero2<C>();
  for (int64_t jb = j0 + (int64_t)s * W; jb < j1; jb += (int64_t)S * W) {
    const int n = (int)min((int64_t)W, j1 - jb);
    int32_t mc = 0;
    R mk = 0, mm = 0;
    if (li < n) {
      mc = colv[jb + li];
      mk = K[jb + li];
      if (MASS) mm = Mv[jb + li];
    }
    for (int t = 0; t < n; t += U) {
      int32_t B[U];
      R k[U], m[U];
      C xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int src = t + u < n ? t + u : 0;
        B[u] = __shfl(mc, src, W);
        k[u] = __shfl(mk, src, W);
        m[u] = MASS ? __shfl(mm, src, W) : (R)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = (ok && t + u < n) ? x[(int64_t)B[u] * G + p] : zero2<C>();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const R kr = mu * k[u], ki = wr * m[u];
        q.x += kr * xv[u].x - ki * xv[u].y;
        q.y += kr * xv[u].y + ki * xv[u].x;
      }
    }
  }
  return q;
}

// k_mg_step for long rows (same arithmetic, split rows; no early exits: every thread
// reaches every barrier).
template <class R, int PD, bool MASS, int MODE>
__global__ void __launch_bounds__(256) k_mg_step_split(LevelArgs<R> la, Batch b, SplitMap sm,
                                                       const double* __restrict__ lam, double lamc, double ratio,
                                                       ChebStep cs, int first,
                                                       const typename CplxOf<R>::C* __restrict__ xk,
                                                       const typename CplxOf<R>::C* __restrict__ xo,
                                                       const typename CplxOf<R>::C* __restrict__ bb,
                                                       typename CplxOf<R>::C* __restrict__ xn) {
  using C = typename CplxOf<R>::C;
  __shared__ C red[256];
  const int t = threadIdx.x, gs = sm.S * sm.W;
  const int rl = t / gs, s = (t / sm.W) % sm.S, li = t % sm.W;
  const int64_t i = (int64_t)blockIdx.x * sm.RB + rl;
  const bool rowok = i < la.n;
  const bool dir = rowok && la.dmask && la.dmask[i] != 0;
  for (int it = 0; it < sm.iters; ++it) {
    const int p = li + it * sm.UL;
    const bool ok = rowok && li < sm.UL && p < sm.G;
    const int slot = b.act[ok ? p / PD : 0];
    const R wr = MASS ? (R)(b.omega[slot] * (double)la.rho) : (R)0;
    C q = zero2<C>();
    if (rowok && !dir) q = slice_row<R, MASS>(la.col, la.K, la.M, la.mu, wr, sm.W, sm.S, s, li, la.ptr[i], la.ptr[i + 1], xk, sm.G, p, ok);
    red[t] = q;
    __syncthreads();
    if (s == 0 && ok) {
      const int64_t ki = i * sm.G + p;
      if (dir) {
        xn[ki] = zero2<C>();
      } else {
        C qt = zero2<C>();
        for (int k = 0; k < sm.S; ++k) {
          const C v = red[rl * gs + k * sm.W + li];
          qt.x += v.x;
          qt.y += v.y;
        }
        C r = bb[ki];
        r.x -= qt.x;
        r.y -= qt.y;
        if (MODE == MG_RESID) {
          xn[ki] = r;
        } else {
          const double lm_ = lam ? lam[slot] : lamc;
          const R dr = la.mu * la.Kd[i], di = MASS ? wr * la.Md[i] : (R)0;
          const C d = cdiv<R, C>(r, dr, di);
          R a, c;
          if (first) {
            a = 0;
            c = (R)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)));
          } else {
            a = (R)(cs.rcur * cs.rprev);
            c = (R)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
          }
          const C xv = xk[ki];
          const C xv0 = (xo && !first) ? xo[ki] : zero2<C>();
          C o;
          o.x = xv.x + a * (xv.x - xv0.x) + c * d.x;
          o.y = xv.y + a * (xv.y - xv0.y) + c * d.y;
          xn[ki] = o;
        }
      }
    }
    __syncthreads();
  }
}

template <class R>
struct SellArgs {
  int64_t nslot;
  const int64_t* off;
  const int32_t* row;
  const int32_t* col;
  const R *K, *M;  // M null: no mass term
};

// Lanes of the sliced-row kernels: W lanes per row (a power of two >= the batch's
// systems, at most 64), each lane one system's PD components; 64 / W rows per wavefront.
struct SellMap {
  int G, W, R;
};
inline SellMap sell_map(int nact, int PD) {
  int W = 1;
  while (W < nact && W < 64) W <<= 1;
  return {nact * PD, W, 64 / W};
}

// k_mg_step on level 0 in sliced rows: same arithmetic, one lane per (row, system)
// accumulating the row's PD components; entry t of the wavefront's rows is one
// contiguous load of column indices and of each value array.
template <class R, int PD, bool MASS, int MODE>
__global__ void __launch_bounds__(256) k_mg_step_sell(LevelArgs<R> la, SellArgs<R> sa, Batch b, SellMap sm,
                                                      const double* __restrict__ lam, double lamc, double ratio,
                                                      ChebStep cs, int first,
                                                      const typename CplxOf<R>::C* __restrict__ xk,
                                                      const typename CplxOf<R>::C* __restrict__ xo,
                                                      const typename CplxOf<R>::C* __restrict__ bb,
                                                      typename CplxOf<R>::C* __restrict__ xn) {
  using C = typename CplxOf<R>::C;
  constexpr int U = 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * sm.R + lane / sm.W;
  if (q >= sa.nslot) return;
  const int32_t i = sa.row[q];
  if (i < 0) return;
  const int64_t sl = q / SELL_C, e0 = sa.off[sl] + q % SELL_C;
  const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
  const bool dir = la.dmask && la.dmask[i] != 0;
  for (int si = lane & (sm.W - 1); si < b.nact; si += sm.W) {
    const int slot = b.act[si];
    const int64_t o = (int64_t)i * sm.G + si * PD;
    if (dir) {
#pragma unroll
      for (int d = 0; d < PD; ++d) xn[o + d] = zero2<C>();
      continue;
    }
    const R wr = MASS ? (R)(b.omega[slot] * (double)la.rho) : (R)0;
    const C* __restrict__ xs = xk + si * PD;
    C acc[PD];
#pragma unroll
    for (int d = 0; d < PD; ++d) acc[d] = zero2<C>();
    for (int t = 0; t < len; t += U) {
      int32_t c[U];
      R k[U], m[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool v = t + u < len;
        const int64_t e = e0 + (int64_t)(t + u) * SELL_C;
        c[u] = v ? sa.col[e] : -1;
        k[u] = v ? sa.K[e] : (R)0;
        m[u] = (MASS && v) ? sa.M[e] : (R)0;
      }
      C xv[U][PD];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int d = 0; d < PD; ++d) xv[u][d] = c[u] >= 0 ? xs[(int64_t)c[u] * sm.G + d] : zero2<C>();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const R kr = la.mu * k[u], ki = wr * m[u];
#pragma unroll
        for (int d = 0; d < PD; ++d) {
          acc[d].x += kr * xv[u][d].x - ki * xv[u][d].y;
          acc[d].y += kr * xv[u][d].y + ki * xv[u][d].x;
        }
      }
    }
    const R dr = la.mu * la.Kd[i], di = MASS ? wr * la.Md[i] : (R)0;
    const double lm_ = lam ? lam[slot] : lamc;
    R a = 0, cc = 0;
    if (MODE == MG_STEP) {
      if (first) {
        cc = (R)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)));
      } else {
        a = (R)(cs.rcur * cs.rprev);
        cc = (R)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
      }
    }
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      C r = bb[o + d];
      r.x -= acc[d].x;
      r.y -= acc[d].y;
      if (MODE == MG_RESID) {
        xn[o + d] = r;
        continue;
      }
      const C dv = cdiv<R, C>(r, dr, di);
      const C xv = xk[o + d];
      const C xv0 = (xo && !first) ? xo[o + d] : zero2<C>();
      C w;
      w.x = xv.x + a * (xv.x - xv0.x) + cc * dv.x;
      w.y = xv.y + a * (xv.y - xv0.y) + cc * dv.y;
      xn[o + d] = w;
    }
  }
}

// k_mg_step on level 0 in sliced rows with two (system, component) pairs per lane
// (FP32, an even number G of pairs per row): a row's group of W lanes gathers a
// column's G values with one 16-byte load per lane, so a wavefront gathers 64 / W
// rows' values in one instruction. Same arithmetic per pair as k_mg_step_sell.
template <int PD, bool MASS, int MODE>
__global__ void __launch_bounds__(256) k_mg_step_sell2(LevelArgs<float> la, SellArgs<float> sa, Batch b, SellMap sm,
                                                       const double* __restrict__ lam, double lamc, double ratio,
                                                       ChebStep cs, int first, const float2* __restrict__ xk,
                                                       const float2* __restrict__ xo, const float2* __restrict__ bb,
                                                       float2* __restrict__ xn) {
  constexpr int U = 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * sm.R + lane / sm.W;
  if (q >= sa.nslot) return;
  const int32_t i = sa.row[q];
  if (i < 0) return;
  const int64_t sl = q / SELL_C, e0 = sa.off[sl] + q % SELL_C;
  const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
  const bool dir = la.dmask && la.dmask[i] != 0;
  const int G = sm.G;
  for (int p0 = 2 * (lane & (sm.W - 1)); p0 < G; p0 += 2 * sm.W) {
    const int64_t o = (int64_t)i * G + p0;
    if (dir) {
      *reinterpret_cast<float4*>(xn + o) = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    const int slot0 = b.act[p0 / PD], slot1 = b.act[(p0 + 1) / PD];
    const float w0 = MASS ? (float)(b.omega[slot0] * (double)la.rho) : 0.f;
    const float w1 = MASS ? (float)(b.omega[slot1] * (double)la.rho) : 0.f;
    float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
    const float2* __restrict__ xs = xk + p0;
    for (int t = 0; t < len; t += U) {
      int32_t c[U];
      float k[U], m[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool v = t + u < len;
        const int64_t e = e0 + (int64_t)(t + u) * SELL_C;
        c[u] = v ? sa.col[e] : -1;
        k[u] = v ? sa.K[e] : 0.f;
        m[u] = (MASS && v) ? sa.M[e] : 0.f;
      }
      float4 xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        xv[u] = c[u] >= 0 ? *reinterpret_cast<const float4*>(xs + (int64_t)c[u] * G) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const float kr = la.mu * k[u], ki0 = w0 * m[u], ki1 = w1 * m[u];
        a0.x += kr * xv[u].x - ki0 * xv[u].y;
        a0.y += kr * xv[u].y + ki0 * xv[u].x;
        a1.x += kr * xv[u].z - ki1 * xv[u].w;
        a1.y += kr * xv[u].w + ki1 * xv[u].z;
      }
    }
    const float4 bv = *reinterpret_cast<const float4*>(bb + o);
    float2 r0 = make_float2(bv.x - a0.x, bv.y - a0.y), r1 = make_float2(bv.z - a1.x, bv.w - a1.y);
    if (MODE == MG_RESID) {
      *reinterpret_cast<float4*>(xn + o) = make_float4(r0.x, r0.y, r1.x, r1.y);
      continue;
    }
    const float4 xv = *reinterpret_cast<const float4*>(xk + o);
    const float4 x0 = (xo && !first) ? *reinterpret_cast<const float4*>(xo + o) : make_float4(0.f, 0.f, 0.f, 0.f);
    float4 w;
    {
      const double lm_ = lam ? lam[slot0] : lamc;
      const float dr = la.mu * la.Kd[i], di = MASS ? w0 * la.Md[i] : 0.f;
      const float2 d = cdiv<float, float2>(r0, dr, di);
      const float a = first ? 0.f : (float)(cs.rcur * cs.rprev);
      const float cc = first ? (float)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)))
                             : (float)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
      w.x = xv.x + a * (xv.x - x0.x) + cc * d.x;
      w.y = xv.y + a * (xv.y - x0.y) + cc * d.y;
    }
    {
      const double lm_ = lam ? lam[slot1] : lamc;
      const float dr = la.mu * la.Kd[i], di = MASS ? w1 * la.Md[i] : 0.f;
      const float2 d = cdiv<float, float2>(r1, dr, di);
      const float a = first ? 0.f : (float)(cs.rcur * cs.rprev);
      const float cc = first ? (float)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)))
                             : (float)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
      w.z = xv.z + a * (xv.z - x0.z) + cc * d.x;
      w.w = xv.w + a * (xv.w - x0.w) + cc * d.y;
    }
    *reinterpret_cast<float4*>(xn + o) = w;
  }
}

// a[act[k]] = 0 for the batch's slots
__global__ void k_zero_slots(double* a, const int* act, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[act[k]] = 0.0;
}

// k_mg_bound on level 0 in sliced rows: one lane per (row, system), the same sums in
// the same entry order, FP64 accumulation of the sliced values (FP32 values on the
// mixed path). The blocks stride over the row blocks; each lane keeps the largest ratio
// of its system over the rows it visits, the wavefront reduces over the lanes of the
// same system (lane mod W), and one lane per system issues the atomic. A maximum does
// not depend on the order, so the bound is the same as with one atomic per (row, system),
// without tens of millions of atomics on a few addresses. Systems beyond the W lanes of
// a row are taken in further passes of W.
template <class R>
__global__ void __launch_bounds__(256) k_mg_bound_sell(LevelArgs<double> la, SellArgs<R> sa, Batch b, int W, int RW,
                                                       unsigned long long* __restrict__ out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t nrb = (sa.nslot + 4 * RW - 1) / (4 * RW);
  for (int s0 = 0; s0 < b.nact; s0 += W) {
    const int si = s0 + (lane & (W - 1));
    const int slot = si < b.nact ? b.act[si] : -1;
    const double wr = slot >= 0 ? b.omega[slot] * la.rho : 0.0;
    double vmax = 0.0;
    for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
      const int64_t q = (rb * 4 + wave) * RW + lane / W;
      if (slot < 0 || q >= sa.nslot) continue;
      const int32_t i = sa.row[q];
      if (i < 0 || (la.dmask && la.dmask[i] != 0)) continue;
      const int64_t sl = q / SELL_C, e0 = sa.off[sl] + q % SELL_C;
      const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
      double sum = 0.0;
      for (int t = 0; t < len; t += 4) {
        int32_t c[4];
        double k[4], m[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool v = t + u < len;
          const int64_t e = e0 + (int64_t)(t + u) * SELL_C;
          c[u] = v ? sa.col[e] : -1;
          k[u] = v ? (double)sa.K[e] : 0.0;
          m[u] = v ? (double)sa.M[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (c[u] < 0 || (la.dmask && la.dmask[c[u]] != 0)) continue;
          const double re = la.mu * k[u], im = wr * m[u];
          sum += sqrt(re * re + im * im);
        }
      }
      const double dr = la.mu * la.Kd[i], di = wr * la.Md[i];
      vmax = fmax(vmax, sum / sqrt(dr * dr + di * di));
    }
    // every lane reaches this point; offsets of W and above keep lane mod W
    for (int off = W; off < 64; off <<= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    if (lane < W && slot >= 0) atomicMax(&out[slot], (unsigned long long)__double_as_longlong(vmax));
  }
}

// Value of lane U of each group of four lanes (DPP quad broadcast).
template <int U>
__device__ __forceinline__ int quad_bcast(int v) {
  return __builtin_amdgcn_mov_dpp(v, U * 0x55, 0xF, 0xF, false);
}
template <int U>
__device__ __forceinline__ float quad_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), U * 0x55, 0xF, 0xF, false));
}

// k_mg_step_sell2 for rows of 6 or 8 pairs (four lanes per row): the four lanes of a
// row load four consecutive entries' (column, K, M) at once and share them by quad
// broadcasts, so a wavefront issues one index and value load per four entries.
template <int PD, bool MASS, int MODE>
__global__ void __launch_bounds__(256) k_mg_step_sell4(LevelArgs<float> la, SellArgs<float> sa, Batch b, SellMap sm,
                                                       const double* __restrict__ lam, double lamc, double ratio,
                                                       ChebStep cs, int first, const float2* __restrict__ xk,
                                                       const float2* __restrict__ xo, const float2* __restrict__ bb,
                                                       float2* __restrict__ xn) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (row_block() * 4 + wave) * 16 + lane / 4;  // sm.W == 4: 16 rows per wavefront
  if (q >= sa.nslot) return;
  const int32_t i = sa.row[q];
  if (i < 0) return;  // uniform over the four lanes of the row
  const int64_t sl = q / SELL_C, e0 = sa.off[sl] + q % SELL_C;
  const int len = (int)((sa.off[sl + 1] - sa.off[sl]) / SELL_C);
  const bool dir = la.dmask && la.dmask[i] != 0;
  const int G = sm.G, li = lane & 3, p0 = 2 * li;
  const bool act = p0 < G;
  const int64_t o = (int64_t)i * G + p0;
  if (dir) {
    if (act) *reinterpret_cast<float4*>(xn + o) = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const int slot0 = b.act[act ? p0 / PD : 0], slot1 = b.act[act ? (p0 + 1) / PD : 0];
  const float w0 = MASS ? (float)(b.omega[slot0] * (double)la.rho) : 0.f;
  const float w1 = MASS ? (float)(b.omega[slot1] * (double)la.rho) : 0.f;
  float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
  const float2* __restrict__ xs = xk + p0;
  for (int t = 0; t < len; t += 8) {
    int32_t cl[2];
    float kl[2], ml[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bool v = t + 4 * h + li < len;
      const int64_t e = e0 + (int64_t)(t + 4 * h + li) * SELL_C;
      cl[h] = v ? sa.col[e] : -1;
      kl[h] = v ? sa.K[e] : 0.f;
      ml[h] = (MASS && v) ? sa.M[e] : 0.f;
    }
    int32_t c[8];
    float k[8], m[8];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      c[4 * h + 0] = quad_bcast<0>(cl[h]);
      c[4 * h + 1] = quad_bcast<1>(cl[h]);
      c[4 * h + 2] = quad_bcast<2>(cl[h]);
      c[4 * h + 3] = quad_bcast<3>(cl[h]);
      k[4 * h + 0] = quad_bcast<0>(kl[h]);
      k[4 * h + 1] = quad_bcast<1>(kl[h]);
      k[4 * h + 2] = quad_bcast<2>(kl[h]);
      k[4 * h + 3] = quad_bcast<3>(kl[h]);
      if (MASS) {
        m[4 * h + 0] = quad_bcast<0>(ml[h]);
        m[4 * h + 1] = quad_bcast<1>(ml[h]);
        m[4 * h + 2] = quad_bcast<2>(ml[h]);
        m[4 * h + 3] = quad_bcast<3>(ml[h]);
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) m[4 * h + u] = 0.f;
      }
    }
    float4 xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      xv[u] = (act && c[u] >= 0) ? *reinterpret_cast<const float4*>(xs + (int64_t)c[u] * G)
                                 : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float kr = la.mu * k[u], ki0 = w0 * m[u], ki1 = w1 * m[u];
      a0.x += kr * xv[u].x - ki0 * xv[u].y;
      a0.y += kr * xv[u].y + ki0 * xv[u].x;
      a1.x += kr * xv[u].z - ki1 * xv[u].w;
      a1.y += kr * xv[u].w + ki1 * xv[u].z;
    }
  }
  if (!act) return;
  const float4 bv = *reinterpret_cast<const float4*>(bb + o);
  float2 r0 = make_float2(bv.x - a0.x, bv.y - a0.y), r1 = make_float2(bv.z - a1.x, bv.w - a1.y);
  if (MODE == MG_RESID) {
    *reinterpret_cast<float4*>(xn + o) = make_float4(r0.x, r0.y, r1.x, r1.y);
    return;
  }
  const float4 xv = *reinterpret_cast<const float4*>(xk + o);
  const float4 x0 = (xo && !first) ? *reinterpret_cast<const float4*>(xo + o) : make_float4(0.f, 0.f, 0.f, 0.f);
  const float a = first ? 0.f : (float)(cs.rcur * cs.rprev);
  float4 w;
  {
    const double lm_ = lam ? lam[slot0] : lamc;
    const float dr = la.mu * la.Kd[i], di = MASS ? w0 * la.Md[i] : 0.f;
    const float2 d = cdiv<float, float2>(r0, dr, di);
    const float cc = first ? (float)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)))
                           : (float)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
    w.x = xv.x + a * (xv.x - x0.x) + cc * d.x;
    w.y = xv.y + a * (xv.y - x0.y) + cc * d.y;
  }
  {
    const double lm_ = lam ? lam[slot1] : lamc;
    const float dr = la.mu * la.Kd[i], di = MASS ? w1 * la.Md[i] : 0.f;
    const float2 d = cdiv<float, float2>(r1, dr, di);
    const float cc = first ? (float)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)))
                           : (float)(2.0 * cs.rcur / (0.5 * lm_ * (1.0 - 1.0 / ratio)));
    w.z = xv.z + a * (xv.z - x0.z) + cc * d.x;
    w.w = xv.w + a * (xv.w - x0.w) + cc * d.y;
  }
  *reinterpret_cast<float4*>(xn + o) = w;
}

// k_mg_restrict for long restriction rows.
template <class R, int PD, bool MASS>
__global__ void __launch_bounds__(256) k_mg_restrict_split(XferArgs<R> rt, LevelArgs<R> lc, Batch b, SplitMap sm,
                                                           const double* __restrict__ lam, double lamc, double ratio,
                                                           const typename CplxOf<R>::C* __restrict__ r,
                                                           typename CplxOf<R>::C* __restrict__ bc,
                                                           typename CplxOf<R>::C* __restrict__ xc) {
  using C = typename CplxOf<R>::C;
  __shared__ C red[256];
  const int t = threadIdx.x, gs = sm.S * sm.W;
  const int rl = t / gs, s = (t / sm.W) % sm.S, li = t % sm.W;
  const int64_t I = (int64_t)blockIdx.x * sm.RB + rl;
  const bool rowok = I < rt.n;
  for (int it = 0; it < sm.iters; ++it) {
    const int p = li + it * sm.UL;
    const bool ok = rowok && li < sm.UL && p < sm.G;
    C q = zero2<C>();
    if (rowok) q = slice_row<R, false>(rt.col, rt.v, rt.v, (R)1, (R)0, sm.W, sm.S, s, li, rt.ptr[I], rt.ptr[I + 1], r, sm.G, p, ok);
    red[t] = q;
    __syncthreads();
    if (s == 0 && ok) {
      C acc = zero2<C>();
      for (int k = 0; k < sm.S; ++k) {
        const C v = red[rl * gs + k * sm.W + li];
        acc.x += v.x;
        acc.y += v.y;
      }
      const int slot = b.act[p / PD];
      const R wr = MASS ? (R)(b.omega[slot] * (double)lc.rho) : (R)0;
      const double lm_ = lam ? lam[slot] : lamc;
      const R dr = lc.mu * lc.Kd[I], di = MASS ? wr * lc.Md[I] : (R)0;
      const C d = cdiv<R, C>(acc, dr, di);
      const R c = (R)(1.0 / (0.5 * lm_ * (1.0 + 1.0 / ratio)));
      const int64_t ki = I * sm.G + p;
      bc[ki] = acc;
      C o;
      o.x = c * d.x;
      o.y = c * d.y;
      xc[ki] = o;
    }
    __syncthreads();
  }
}

// Coarsest level: x[i][p] = sum_j Ainv_s[i][j] b[j][p] with the dense inverse of the
// lane's system (inverses `ist` apart; ist = 0: one inverse for all systems).
template <class C, int PD>
__global__ void __launch_bounds__(256) k_mg_dense(const C* __restrict__ inv, int64_t ist, int64_t n, Batch b, int G,
                                                  const C* __restrict__ bb, C* __restrict__ x) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * G) return;
  const int64_t i = idx / G;
  const int p = (int)(idx - i * G);
  const C* __restrict__ a = inv + (ist ? (int64_t)b.act[p / PD] * ist : 0) + i * n;
  C acc = zero2<C>();
  for (int64_t j = 0; j < n; ++j) {
    const C m = a[j], v = bb[j * G + p];
    acc.x += m.x * v.x - m.y * v.y;
    acc.y += m.x * v.y + m.y * v.x;
  }
  x[idx] = acc;
}

// Dense inverse of the coarsest velocity operator mu K + j w rho M of system blockIdx.x
// of the batch (FP64 Gauss-Jordan without pivoting in the slot's n x n block, plus an
// FP32 copy when inv32 is given).
__global__ void __launch_bounds__(1024) k_mg_cinv(LevelArgs<double> la, Batch b, double2* __restrict__ inv,
                                                  float2* __restrict__ inv32) {
  __shared__ double2 rk[MG_COARSE_MAX], fk[MG_COARSE_MAX];
  const int slot = b.act[blockIdx.x];
  const int64_t n = la.n;
  double2* __restrict__ a = inv + (int64_t)slot * n * n;
  const double wr = b.omega[slot] * la.rho;
  for (int64_t q = threadIdx.x; q < n * n; q += blockDim.x) a[q] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    for (int64_t k = la.ptr[i]; k < la.ptr[i + 1]; ++k) {
      double2& e = a[i * n + la.col[k]];
      e.x += la.mu * la.K[k];
      e.y += wr * la.M[k];
    }
  __syncthreads();
  for (int64_t k = 0; k < n; ++k) {
    const double2 pv = a[k * n + k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    if (den == 0.0) continue;  // uniform over the workgroup: a row without couplings stays zero
    const double2 pinv = make_double2(pv.x / den, -pv.y / den);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      const double2 v = j == k ? make_double2(1.0, 0.0) : a[k * n + j];
      rk[j] = make_double2(v.x * pinv.x - v.y * pinv.y, v.x * pinv.y + v.y * pinv.x);
      fk[j] = a[j * n + k];
    }
    __syncthreads();
    for (int64_t q = threadIdx.x; q < n * n; q += blockDim.x) {
      const int64_t i = q / n, j = q - i * n;
      if (i == k) {
        a[q] = rk[j];
      } else {
        const double2 o = j == k ? make_double2(0.0, 0.0) : a[q];
        const double2 f = fk[i], r = rk[j];
        a[q] = make_double2(o.x - (f.x * r.x - f.y * r.y), o.y - (f.x * r.y + f.y * r.x));
      }
    }
    __syncthreads();
  }
  if (inv32)
    for (int64_t q = threadIdx.x; q < n * n; q += blockDim.x)
      inv32[(int64_t)slot * n * n + q] = make_float2((float)a[q].x, (float)a[q].y);
}

template <class R>
LevelArgs<R> level_args(const MgLevel& L, double mu, double rho);
template <>
LevelArgs<double> level_args<double>(const MgLevel& L, double mu, double rho) {
  return {L.n, L.ptr, L.col, L.K, L.M.p, L.Kd, L.M.p ? L.Md.p : nullptr, nullptr, mu, rho};
}
template <>
LevelArgs<float> level_args<float>(const MgLevel& L, double mu, double rho) {
  return {L.n, L.ptr, L.col, L.K32, L.M32.p, L.Kd32, L.M32.p ? L.Md32.p : nullptr, nullptr, (float)mu, (float)rho};
}
template <class R>
XferArgs<R> p_args(const MgLevel& L);
template <>
XferArgs<double> p_args<double>(const MgLevel& L) {
  return {L.n, L.pptr, L.pcol, L.pval};
}
template <>
XferArgs<float> p_args<float>(const MgLevel& L) {
  return {L.n, L.pptr, L.pcol, L.pval32};
}
template <class R>
XferArgs<R> r_args(const MgLevel& L);
template <>
XferArgs<double> r_args<double>(const MgLevel& L) {
  return {L.nc, L.rptr, L.rcol, L.rval};
}
template <>
XferArgs<float> r_args<float>(const MgLevel& L) {
  return {L.nc, L.rptr, L.rcol, L.rval32};
}

// Algorithmic bytes of `launches` smoothing or residual launches on a level: the
// level's pattern and values once, and per pair the gathered input once plus
// `streams` other vectors read or written, per launch.
double level_bytes(int64_t n, int64_t nnz, bool mass, int vb, int64_t pairs, int streams) {
  return (double)nnz * (4.0 + vb * (mass ? 2.0 : 1.0)) + (double)n * (8.0 + vb * (mass ? 2.0 : 1.0)) +
         (double)n * pairs * 2.0 * vb * (1 + streams);
}

// One V-cycle on the levels from `l` down for the pairs of batch b (PD per system):
// nu smoothing steps before and after each coarse correction (post0 > 0: post0 after
// it on level l = 0).
// On entry level l holds its right-hand side in buffer 0 and the first smoothing
// iterate x_1 in buffer 2 (x_k lives in buffer 1 + k % 3; buffer 4 takes the
// residual). Returns the buffer that holds the level's result: 1 + (nu + post) % 3, or 2
// on the coarsest level (its dense inverse applied to buffer 0). With `out` the last
// post-smoothing step of level l writes there instead (same [n][G] layout).
struct CoarseInv {
  const void* inv;  // complex, FP32 or FP64 like the cycle
  int64_t ist;      // elements between the inverses of two slots (0: one for all)
};

// A level in sliced rows with values in precision R; all null (the CSR kernels run)
// when it has no sliced copy or those values were not filled.
template <class R>
SellArgs<R> sell_args(const Sell& S, bool mass) {
  const R* K;
  const R* M;
  if constexpr (sizeof(R) == 4) {
    K = S.K32.p;
    M = S.M32.p;
  } else {
    K = S.K.p;
    M = S.M.p;
  }
  if (!K || (mass && !M)) return {0, nullptr, nullptr, nullptr, nullptr, nullptr};
  return {S.nslot, S.off, S.row, S.col, K, mass ? M : nullptr};
}

template <class R, int PD, bool MASS>
int mg_cycle(const MgHier& H, const std::vector<LevelArgs<R>>& las, const SellArgs<R>& sell0,
             const std::vector<void*>& bufs, const std::vector<const double*>& lams, int l, const Batch& b, int nu,
             int post0, double ratio, CoarseInv coarse, typename CplxOf<R>::C* out, Profiler* prof, hipStream_t s) {
  using C = typename CplxOf<R>::C;
  const LaneMap lm = lane_map(b.nact, PD);
  const int nlev = (int)las.size();
  const LevelArgs<R>& la = las[l];
  C* base = reinterpret_cast<C*>(bufs[l]);
  const int64_t nG = la.n * lm.G;
  auto arr = [&](int k) { return base + (int64_t)k * nG; };
  auto iter = [&](int k) { return arr(1 + k % 3); };
  const double* lam = lams[l];
  const double lamc = H.lv[l].lam;
  const int vb = (int)sizeof(R);
  const int64_t nnz = la.ptr ? H.lv[l].nnz : 0;
  const unsigned nb = row_blocks(la.n, lm);
  // profiler names: velocity (PD > 1) or pressure hierarchy, level 0 or below
  const bool v = PD > 1, z0 = l == 0;
  const char* n_smooth = v ? (z0 ? "k_mgv_smooth0" : "k_mgv_smooth") : (z0 ? "k_mgp_smooth0" : "k_mgp_smooth");
  const char* n_resid = v ? (z0 ? "k_mgv_resid0" : "k_mgv_resid") : (z0 ? "k_mgp_resid0" : "k_mgp_resid");
  const char* n_restr = v ? (z0 ? "k_mgv_restrict0" : "k_mgv_restrict") : "k_mgp_restrict";
  const char* n_prol = v ? (z0 ? "k_mgv_prolong0" : "k_mgv_prolong") : "k_mgp_prolong";
  if (l == nlev - 1) {
    ProfScope ps(prof, s, v ? "k_mgv_dense" : "k_mgp_dense", (double)la.n * la.n * 2.0 * vb * (coarse.ist ? b.nact : 1) +
                                            (double)nG * 4.0 * vb);
    k_mg_dense<C, PD><<<(unsigned)((nG + 255) / 256), 256, 0, s>>>(reinterpret_cast<const C*>(coarse.inv),
                                                                   coarse.ist, la.n, b, lm.G, arr(0), arr(2));
    launch_check(s);
    return 2;
  }
  // one smoothing or residual launch on this level: split rows when they are long
  const SplitMap sm = split_map(lm, la.n ? (double)nnz / (double)la.n : 0.0);
  const unsigned nbs = (unsigned)((la.n + sm.RB - 1) / sm.RB);
  // level 0: the caller's sliced rows; large coarse levels: their own
  const SellArgs<R> sl = l == 0 ? sell0 : sell_args<R>(H.lv[l].sell, MASS);
  const SellMap ssm = sell_map(b.nact, PD);
  const unsigned nbsell = (unsigned)((sl.nslot + 4 * ssm.R - 1) / (4 * ssm.R));
  // two pairs per lane (FP32, even G): W lanes per row cover the G pairs in 16-byte loads
  const bool two = sizeof(R) == 4 && lm.G % 2 == 0;
  SellMap sm2{lm.G, 1, 64};
  while (sm2.W < lm.G / 2 && sm2.W < 64) sm2.W <<= 1;
  sm2.R = 64 / sm2.W;
  const unsigned nbsell2 = (unsigned)((sl.nslot + 4 * sm2.R - 1) / (4 * sm2.R));
  auto step = [&](int mode, ChebStep cs, int first, const C* xk, const C* xo, C* xn) {
    if constexpr (sizeof(R) == 4) {
      if (sl.off && two && sm2.W == 4) {
        if (mode == MG_STEP)
          k_mg_step_sell4<PD, MASS, MG_STEP><<<nbsell2, 256, 0, s>>>(la, sl, b, sm2, lam, lamc, ratio, cs, first,
                                                                      xk, xo, arr(0), xn);
        else
          k_mg_step_sell4<PD, MASS, MG_RESID><<<nbsell2, 256, 0, s>>>(la, sl, b, sm2, lam, lamc, ratio, cs, first,
                                                                       xk, xo, arr(0), xn);
        return;
      }
      if (sl.off && two) {
        if (mode == MG_STEP)
          k_mg_step_sell2<PD, MASS, MG_STEP><<<nbsell2, 256, 0, s>>>(la, sl, b, sm2, lam, lamc, ratio, cs, first,
                                                                      xk, xo, arr(0), xn);
        else
          k_mg_step_sell2<PD, MASS, MG_RESID><<<nbsell2, 256, 0, s>>>(la, sl, b, sm2, lam, lamc, ratio, cs, first,
                                                                       xk, xo, arr(0), xn);
        return;
      }
    }
    if (sl.off) {
      if (mode == MG_STEP)
        k_mg_step_sell<R, PD, MASS, MG_STEP><<<nbsell, 256, 0, s>>>(la, sl, b, ssm, lam, lamc, ratio, cs, first,
                                                                     xk, xo, arr(0), xn);
      else
        k_mg_step_sell<R, PD, MASS, MG_RESID><<<nbsell, 256, 0, s>>>(la, sl, b, ssm, lam, lamc, ratio, cs, first,
                                                                      xk, xo, arr(0), xn);
    } else if (sm.S > 1) {
      if (mode == MG_STEP)
        k_mg_step_split<R, PD, MASS, MG_STEP><<<nbs, 256, 0, s>>>(la, b, sm, lam, lamc, ratio, cs, first, xk, xo,
                                                                   arr(0), xn);
      else
        k_mg_step_split<R, PD, MASS, MG_RESID><<<nbs, 256, 0, s>>>(la, b, sm, lam, lamc, ratio, cs, first, xk, xo,
                                                                    arr(0), xn);
    } else {
      if (mode == MG_STEP)
        k_mg_step<R, PD, MASS, MG_STEP><<<nb, 256, 0, s>>>(la, b, lm, lam, lamc, ratio, cs, first, xk, xo, arr(0),
                                                            xn);
      else
        k_mg_step<R, PD, MASS, MG_RESID><<<nb, 256, 0, s>>>(la, b, lm, lam, lamc, ratio, cs, first, xk, xo, arr(0),
                                                             xn);
    }
  };
  if (nu > 1) {
    ProfScope ps(prof, s, n_smooth, level_bytes(la.n, nnz, MASS, vb, lm.G, 2) * (nu - 1), nu - 1);
    for (int k = 1; k < nu; ++k)
      step(MG_STEP, cheb_step(ratio, k), 0, iter(k), k == 1 ? nullptr : iter(k - 1), iter(k + 1));
  }
  {
    ProfScope ps(prof, s, n_resid, level_bytes(la.n, nnz, MASS, vb, lm.G, 1));
    step(MG_RESID, ChebStep{0, 0}, 0, iter(nu), nullptr, arr(4));
  }
  const LevelArgs<R>& lc = las[l + 1];
  C* cb = reinterpret_cast<C*>(bufs[l + 1]);
  const int64_t ncG = lc.n * lm.G;
  {
    const XferArgs<R> rt = r_args<R>(H.lv[l]);
    const double tb = (double)H.lv[l].pval.n * (4.0 + vb) + (double)lc.n * 8.0 + (double)la.n * lm.G * 2.0 * vb +
                      (double)lc.n * lm.G * 4.0 * vb;
    ProfScope ps(prof, s, n_restr, tb);
    const SplitMap smr = split_map(lm, lc.n ? (double)H.lv[l].pval.n / (double)lc.n : 0.0);
    if (smr.S > 1)
      k_mg_restrict_split<R, PD, MASS><<<(unsigned)((lc.n + smr.RB - 1) / smr.RB), 256, 0, s>>>(
          rt, lc, b, smr, lams[l + 1], H.lv[l + 1].lam, ratio, arr(4), cb, cb + 2 * ncG);
    else
      k_mg_restrict<R, PD, MASS><<<row_blocks(lc.n, lm), 256, 0, s>>>(rt, lc, b, lm, lams[l + 1], H.lv[l + 1].lam,
                                                                     ratio, arr(4), cb, cb + 2 * ncG);
  }
  launch_check(s);
  const int kres =
      mg_cycle<R, PD, MASS>(H, las, sell0, bufs, lams, l + 1, b, nu, 0, ratio, coarse, nullptr, prof, s);
  {
    const double tb = (double)H.lv[l].pval.n * (4.0 + vb) + (double)la.n * 8.0 + (double)la.n * lm.G * 4.0 * vb +
                      (double)lc.n * lm.G * 2.0 * vb;
    ProfScope ps(prof, s, n_prol, tb);
    k_mg_prolong<R><<<nb, 256, 0, s>>>(p_args<R>(H.lv[l]), lm, cb + (int64_t)kres * ncG, iter(nu));
  }
  // post-smoothing: post0 steps on level 0 when given, else nu
  const int npost = (l == 0 && post0 > 0) ? post0 : nu;
  {
    ProfScope ps(prof, s, n_smooth, level_bytes(la.n, nnz, MASS, vb, lm.G, 2) * npost, npost);
    for (int j = 1; j <= npost; ++j)
      step(MG_STEP, cheb_step(ratio, j - 1), j == 1 ? 1 : 0, iter(nu + j - 1), j == 1 ? nullptr : iter(nu + j - 2),
           (j == npost && out) ? out : iter(nu + j));
  }
  launch_check(s);
  return 1 + (nu + npost) % 3;
}

// z[slot][i*D + c] = buf[i*G + p] (p = si*D + c): the interleaved result in the
// system-major layout of the Krylov vectors.
template <class C, class ZT, int D>
__global__ void k_il_to_sys(const C* __restrict__ buf, int64_t n, const int* __restrict__ act, int nact,
                            SV<ZT> z) {
  const int64_t G = (int64_t)nact * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * G;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / G;
    const int p = (int)(idx - i * G);
    const C v = buf[idx];
    ZT o;
    o.x = v.x;
    o.y = v.y;
    z.at(act[p / D])[i * D + p % D] = o;
  }
}

// Schur block of the systems with w != 0: z_p = -(mu Mp^-1 insc v_p + j w rho x),
// x = L^-1 insc v_p from the pressure cycle (interleaved [nv][nact]); FP64 combination.
template <class C, class VI>
__global__ void k_p_combine(const C* __restrict__ x, int64_t nv, int64_t DN, Batch b, const double* __restrict__ Mp,
                            double mu, double rho, SV<VI> v, VArg z) {
  const int G = b.nact;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < nv * G;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / G;
    const int si = (int)(idx - i * G);
    const int slot = b.act[si];
    const double w = schur_w(b, slot);
    if (w == 0.0) continue;  // final already (no Laplacian term)
    const double sc = b.insc ? b.insc[(int64_t)slot * b.insc_st + b.insc_idx] : 1.0;
    const VI vv = v.at(slot)[DN + i];
    const double vx = sc * (double)vv.x, vy = sc * (double)vv.y;
    const C xl = x[idx];
    const double wr = w * rho, im = mu / Mp[i];
    z.at(slot)[DN + i] = make_double2(-(im * vx - wr * (double)xl.y), -(im * vy + wr * (double)xl.x));
  }
}

template <class R>
std::vector<LevelArgs<R>> vel_levels(scvs_mesh m) {
  const MgHier& H = m->mg->vel;
  std::vector<LevelArgs<R>> las(H.lv.size());
  if constexpr (sizeof(R) == 4)
    las[0] = {m->n2, m->rowptr, m->col, m->Ks32, m->M32, m->Kd32, m->Md32, m->dmask, (float)m->mu, (float)m->rho};
  else
    las[0] = {m->n2, m->rowptr, m->col, m->Ks, m->M, m->Kd, m->Md, m->dmask, m->mu, m->rho};
  for (size_t l = 1; l < H.lv.size(); ++l) las[l] = level_args<R>(H.lv[l], m->mu, m->rho);
  return las;
}

template <class R>
std::vector<LevelArgs<R>> pres_levels(scvs_mesh m) {
  const MgHier& H = m->mg->pres;
  std::vector<LevelArgs<R>> las(H.lv.size());
  for (size_t l = 0; l < H.lv.size(); ++l) las[l] = level_args<R>(H.lv[l], 1.0, 0.0);
  return las;
}


template <class R, int D>
void vel_cycle(scvs_mesh m, const Batch& b, const PrecondArgs& pa, void* zil, SV<typename CplxOf<R>::C> z,
               hipStream_t s) {
  using C = typename CplxOf<R>::C;
  const MgHier& H = m->mg->vel;
  const auto las = vel_levels<R>(m);
  const SellArgs<R> s0 = sell_args<R>(m->s2sell, true);
  std::vector<void*> bufs(H.lv.size());
  std::vector<const double*> lams(H.lv.size());
  for (size_t l = 0; l < H.lv.size(); ++l) {
    bufs[l] = pa.mg.v[l];
    lams[l] = pa.mg.vlam + l * pa.mg.slots;
  }
  Profiler* prof = &m->ctx->prof;
  const int64_t nc = H.lv.back().n;
  const CoarseInv ci{pa.mg.vinv, nc * nc};
  const int k = mg_cycle<R, D, true>(H, las, s0, bufs, lams, 0, b, pa.mg_nu, pa.mg_post0, pa.mg_ratio, ci,
                                     reinterpret_cast<C*>(zil), prof, s);
  if (!zil) {
    const int64_t G = (int64_t)b.nact * D;
    const C* res = reinterpret_cast<C*>(pa.mg.v[0]) + (int64_t)k * m->n2 * G;
    ProfScope ps(prof, s, "k_il_to_sys", (double)m->n2 * G * 2.0 * sizeof(C));
    k_il_to_sys<C, C, D><<<1024, 256, 0, s>>>(res, m->n2, b.act, b.nact, z);
    launch_check(s);
  }
}

template <class R, class VI>
void pres_cycle(scvs_mesh m, const Batch& b, const PrecondArgs& pa, SV<VI> v, VArg z, hipStream_t s) {
  using C = typename CplxOf<R>::C;
  const MgHier& H = m->mg->pres;
  const auto las = pres_levels<R>(m);
  const SellArgs<R> s0 = sell_args<R>(H.sell0, false);
  std::vector<void*> bufs(H.lv.size());
  std::vector<const double*> lams(H.lv.size(), nullptr);
  for (size_t l = 0; l < H.lv.size(); ++l) bufs[l] = pa.mg.p[l];
  Profiler* prof = &m->ctx->prof;
  const CoarseInv ci{sizeof(R) == 4 ? (const void*)H.cinv32.p : (const void*)H.cinv.p, 0};
  const int k = mg_cycle<R, 1, false>(H, las, s0, bufs, lams, 0, b, pa.mg_nu, 0, pa.mg_ratio, ci, nullptr, prof, s);
  const C* res = reinterpret_cast<C*>(pa.mg.p[0]) + (int64_t)k * m->nv * b.nact;
  ProfScope ps(prof, s, "k_p_combine", (double)m->nv * (8.0 + b.nact * (sizeof(C) + sizeof(VI) + 16.0)));
  k_p_combine<C, VI><<<1024, 256, 0, s>>>(res, m->nv, (int64_t)m->dim * m->n2, b, m->Mp, m->mu, m->rho, v, z);
  launch_check(s);
}

}  // namespace

// Device temporaries of the levels below level 0 (level 0 uses the preconditioner's own
// temporaries), complex elements of `esize` bytes: 5 arrays per level for `slots` systems.
size_t mg_buffer_bytes(scvs_mesh m, int slots, size_t esize, bool vel, bool pres) {
  size_t t = 0;
  const int D = m->dim;
  if (vel)
    for (size_t l = 1; l < m->mg->vel.lv.size(); ++l) t += 5 * (size_t)m->mg->vel.lv[l].n * slots * D * esize + 256;
  if (pres)
    for (size_t l = 1; l < m->mg->pres.lv.size(); ++l) t += 5 * (size_t)m->mg->pres.lv[l].n * slots * esize + 256;
  return t;
}

void mg_assign(scvs_mesh m, int slots, size_t esize, bool vel, bool pres, char* base, void* vel0, void* pres0,
               double* vlam, MgBufs& out) {
  const int D = m->dim;
  out.slots = slots;
  out.vlam = vlam;
  auto take = [&](size_t bytes) {
    char* p = base;
    base += (bytes + 255) / 256 * 256;
    return (void*)p;
  };
  for (auto& p : out.v) p = nullptr;
  for (auto& p : out.p) p = nullptr;
  if (vel) {
    SCVS_REQUIRE(m->mg->vel.lv.size() <= (size_t)MG_MAXLEV, SCVS_E_CAPACITY, "too many multigrid levels");
    out.v[0] = vel0;
    for (size_t l = 1; l < m->mg->vel.lv.size(); ++l) out.v[l] = take(5 * (size_t)m->mg->vel.lv[l].n * slots * D * esize);
  }
  if (pres) {
    SCVS_REQUIRE(m->mg->pres.lv.size() <= (size_t)MG_MAXLEV, SCVS_E_CAPACITY, "too many multigrid levels");
    out.p[0] = pres0;
    for (size_t l = 1; l < m->mg->pres.lv.size(); ++l) out.p[l] = take(5 * (size_t)m->mg->pres.lv[l].n * slots * esize);
  }
}

// Sliced-row values of level 0 in the cycle's precision (FP32 when f32), for the
// hierarchies in use; once per assembly and precision, outside any graph capture.
void mg_sell_values(scvs_mesh m, bool f32, bool vel, bool pres, hipStream_t s) {
  if (vel) s2sell_setup(m, f32, !f32, s);
  if (pres) {
    Sell& S = m->mg->pres.sell0;
    const MgLevel& L0 = m->mg->pres.lv[0];
    if (f32 && !S.K32.p) sell_values<float>(S, m->lp_ptr, L0.K32.p, S.K32, s);
    if (!f32 && !S.K.p) sell_values<double>(S, m->lp_ptr, L0.K.p, S.K, s);
  }
}

int mg_levels(scvs_mesh m, bool vel) { return (int)(vel ? m->mg->vel.lv.size() : m->mg->pres.lv.size()); }

// Per system of the batch: the Gershgorin bounds of every velocity level into
// lam[l * slots + slot] and the dense inverse of the coarsest level into
// inv[slot] (n_c x n_c, FP64) and, when given, its FP32 copy inv32[slot].
void mg_prepare(scvs_mesh m, const Batch& b, double* lam, int slots, double2* inv, float2* inv32, hipStream_t s) {
  const MgHier& H = m->mg->vel;
  const LaneMap lm = lane_map(b.nact, 1);
  const auto las = vel_levels<double>(m);
  int W = 1;
  while (W < b.nact && W < 64) W <<= 1;
  const int RW = 64 / W;
  const SellArgs<float> s32 = sell_args<float>(m->s2sell, true);
  const SellArgs<double> s64 = sell_args<double>(m->s2sell, true);
  for (size_t l = 0; l < H.lv.size(); ++l) {
    // only the listed slots: other slots of the pool may be running
    k_zero_slots<<<(b.nact + 63) / 64, 64, 0, s>>>(lam + l * slots, b.act, b.nact);
    unsigned long long* o = reinterpret_cast<unsigned long long*>(lam + l * slots);
    // level 0 from its sliced rows in the cycle's precision when they are there
    // sliced level 0: at most 2048 blocks striding over the row blocks (one atomic per
    // wavefront and system at the end)
    if (l == 0 && inv32 && s32.off)
      k_mg_bound_sell<float><<<(unsigned)std::min<int64_t>(2048, (s32.nslot + 4 * RW - 1) / (4 * RW)), 256, 0, s>>>(
          las[0], s32, b, W, RW, o);
    else if (l == 0 && !inv32 && s64.off)
      k_mg_bound_sell<double><<<(unsigned)std::min<int64_t>(2048, (s64.nslot + 4 * RW - 1) / (4 * RW)), 256, 0, s>>>(
          las[0], s64, b, W, RW, o);
    else
      k_mg_bound<true><<<row_blocks(las[l].n, lm), 256, 0, s>>>(las[l], b, lm, o);
    launch_check(s);
  }
  ProfScope ps(&m->ctx->prof, s, "k_mg_cinv", 0.0);
  k_mg_cinv<<<(unsigned)b.nact, 1024, 0, s>>>(las.back(), b, inv, inv32);
  launch_check(s);
}

int64_t mg_coarse_rows(scvs_mesh m) { return m->mg->vel.lv.back().n; }

int mg_info(scvs_mesh m, int which, int maxlev, int64_t* rows, int64_t* nnz, int64_t* pnnz) {
  mg_setup(m, m->ctx->stream);
  const MgHier& H = which == 0 ? m->mg->vel : m->mg->pres;
  const int n = (int)H.lv.size();
  for (int l = 0; l < n && l < maxlev; ++l) {
    rows[l] = H.lv[l].n;
    nnz[l] = H.lv[l].nnz;
    pnnz[l] = (int64_t)H.lv[l].pval.n * (H.lv[l].pptr.p != nullptr);
  }
  return n;
}

void mg_velocity(scvs_mesh m, const Batch& b, const PrecondArgs& pa, void* zil, VArg z, hipStream_t s) {
  if (m->dim == 2) {
    if (pa.mixed)
      vel_cycle<float, 2>(m, b, pa, zil, pa.z32, s);
    else
      vel_cycle<double, 2>(m, b, pa, zil, z, s);
  } else {
    if (pa.mixed)
      vel_cycle<float, 3>(m, b, pa, zil, pa.z32, s);
    else
      vel_cycle<double, 3>(m, b, pa, zil, z, s);
  }
}

void mg_pressure(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s) {
  if (pa.mixed)
    pres_cycle<float, double2>(m, b, pa, v, z, s);
  else
    pres_cycle<double, double2>(m, b, pa, v, z, s);
}

void mg_pressure(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg32 v, VArg z, hipStream_t s) {
  if (pa.mixed)
    pres_cycle<float, float2>(m, b, pa, v, z, s);
  else
    pres_cycle<double, float2>(m, b, pa, v, z, s);
}

}  // namespace scvs

// Internal declarations of the SCVS HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <random>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "../../include/scvs.h"

namespace scvs {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

#define SCVS_HIP(call)                                                                \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      (void)hipGetLastError(); /* do not leave a sticky error for later calls */       \
      ::scvs::fail(SCVS_E_HIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    }                                                                                 \
  } while (0)

#define SCVS_REQUIRE(cond, code, msg) \
  do {                                \
    if (!(cond)) ::scvs::fail(code, msg); \
  } while (0)

// Owning device buffer.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      p = nullptr;
      fail(SCVS_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    n = count;
  }
  void zero(hipStream_t s) { SCVS_HIP(hipMemsetAsync(p, 0, n * sizeof(T), s)); }
  void upload(const T* h, size_t count, hipStream_t s) {
    alloc(count);
    if (count) SCVS_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  operator T*() const { return p; }
};

}  // namespace scvs

namespace scvs {
// Event-based per-kernel timing on the launching stream (see scvs_profile_*).
struct Profiler {
  struct Stat {
    int64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes;
    int count;  // launches inside the span
  };
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Pending> pending;
  std::vector<std::pair<std::string, Stat>> stats;
  std::vector<std::pair<std::string, double>> corrections;  // bytes charged for work skipped on the device
  hipEvent_t get();
  void resolve();  // synchronizes, folds pending pairs and byte corrections into stats
  void correct(const char* name, double bytes) {
    if (on) corrections.push_back({name, bytes});
  }
  ~Profiler();
};
// Brackets one launch with events when profiling is on; a scope around `count`
// back-to-back launches of one kernel (no host work between them) times them as one
// span, so its per-launch average includes the gaps between those launches.
class ProfScope {
 public:
  ProfScope(Profiler* p, hipStream_t s, const char* name, double bytes, int count = 1);
  ~ProfScope();

 private:
  Profiler* p_;
  hipStream_t s_;
  size_t idx_ = (size_t)-1;
};
}  // namespace scvs

struct scvs_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream: all work runs here
  hipStream_t capture = nullptr;  // private stream used only to record graphs
  uint64_t mem_cap = 0;           // bytes a solve's Krylov slot pool may take (0: 90% of free memory)
  scvs::Profiler prof;
  // autotuner results, keyed by (mesh id, operator generation, systems, every caller option
  // that the tuner does not choose); only the tuned fields are kept
  struct Tuned {
    int restart, cheb_vel, cheb_pres, mg_smooth;
    double mg_ratio, ms;
  };
  std::map<std::tuple<uint64_t, uint64_t, int64_t, std::string>, Tuned> tuned;
};

constexpr int SCVS_MMAX = 256;  // largest Krylov dimension per cycle

namespace scvs {
// One level of an aggregation multigrid hierarchy (device): its operator pair (K, M;
// M empty for a single-matrix hierarchy) with diagonals, FP32 copies, and the
// transfer to the next coarser level, P (n x nc) and R = P^T (nc x n).
// Sliced rows of an operator for the wide row kernels: rows are ordered by
// length (longest first, ties by index) inside windows of SELL_WIN consecutive rows
// and cut into slices of SELL_C rows; entry t of the r-th row of slice s sits at
// off[s] + t * SELL_C + r, so that one wavefront load of entry t covers SELL_C rows
// in one contiguous run. Rows shorter than their slice are padded with their own
// index and zero values. Values are filled per precision on first use.
// Rows below a split index (the vertex rows of S2) fill the first split_slots slots,
// the others start on a fresh slice, so no slice mixes the two kinds.
constexpr int SELL_C = 32, SELL_WIN = 512;
struct Sell {
  int64_t nslot = 0;          // slices * SELL_C
  int64_t split_slots = 0;    // slots of the rows below the split (a multiple of SELL_C)
  int64_t split_entries = 0;  // their entries (off[split_slots / SELL_C])
  DBuf<int64_t> off;          // [slices + 1]
  DBuf<int32_t> row;          // [nslot] row of each slot, -1 for padding slots
  DBuf<int32_t> col;          // [off[slices]]
  DBuf<float> K32, M32;
  DBuf<double> K, M;
};

struct MgLevel {
  int64_t n = 0, nnz = 0, nc = 0;
  DBuf<int64_t> ptr;
  DBuf<int32_t> col;
  DBuf<double> K, M, Kd, Md;
  DBuf<float> K32, M32, Kd32, Md32;
  DBuf<int64_t> pptr, rptr;
  DBuf<int32_t> pcol, rcol;
  DBuf<double> pval, rval;
  DBuf<float> pval32, rval32;
  double lam = 0.0;  // Gershgorin bound of D^-1 K (single-matrix hierarchies)
  Sell sell;         // levels below 0 with at least MG_SELL_MIN rows: the operator in sliced rows
};
struct MgHier {
  std::vector<MgLevel> lv;
  Sell sell0;  // pressure: level 0 in sliced rows (the velocity's level 0 is the mesh's S2)
  bool mass = false;
  DBuf<double2> cinv;  // single-matrix hierarchies: dense inverse of the coarsest level
  DBuf<float2> cinv32;
};
constexpr int MG_COARSE_MAX = 256;  // rows of the coarsest level (inverted densely)
constexpr int64_t MG_SELL_MIN = 65536;  // coarse levels at least this large also get sliced rows
struct MgData {
  uint64_t gen = ~0ull;  // operator generation it was built for
  MgHier vel;            // lv[0]: the quadratic pattern (transfer only), then P1 and aggregates
  MgHier pres;           // lv[0]: the assembled pressure Laplacian
};
constexpr int MG_MAXLEV = 12;
// Temporaries of one preconditioner application: per level 5 interleaved arrays.
struct MgBufs {
  void* v[MG_MAXLEV] = {};
  void* p[MG_MAXLEV] = {};
  const double* vlam = nullptr;  // [level][slots] per-system velocity bounds
  const void* vinv = nullptr;    // [slots][nc][nc] coarsest velocity inverses (FP32 in mixed mode)
  int slots = 0;
};
}  // namespace scvs

struct scvs_mesh_s {
  scvs_ctx ctx = nullptr;
  uint64_t uid = 0;  // unique per mesh object in this process (never reused, unlike addresses)
  int dim = 0, nvl = 0, nn = 0;  // dim, vertices per cell, quadratic nodes per cell
  int64_t nv = 0, nc = 0, nf = 0, ne = 0, n2 = 0;
  int64_t nnz = 0, nnz21 = 0, nnzv = 0;  // S2 slots, vertex-column slots, slots of vertex rows
  scvs::DBuf<double> xyz, exyz;            // vertex and midside coordinates
  scvs::DBuf<int32_t> cells, c2n, edges, bfaces, btags, fnodes;
  scvs::DBuf<int64_t> vc_ptr;  // vertex -> cells (ascending)
  scvs::DBuf<int32_t> vc;
  scvs::DBuf<int64_t> vn_ptr;  // vertex a -> sorted neighbours b > a (edge list)
  scvs::DBuf<int32_t> vn;
  scvs::DBuf<int64_t> rowptr, rowptr21;
  scvs::DBuf<int32_t> col, nvc;
  scvs::DBuf<int64_t> nf_ptr;  // node -> boundary facets (ascending)
  scvs::DBuf<int32_t> nf_list;
  // assembled values
  scvs::DBuf<double> Ks, M, G, Gt, Kd, Md, Mp;
  scvs::DBuf<float> Ks32, M32, G32, Gt32, Kd32, Md32;  // made on the first mixed-precision solve
  // S2 in sliced rows (vertex rows first): the pattern once per mesh, values per
  // assembly and precision on first use; G on each row's vertex-column prefix in
  // slices of their own (s2_goff, D values per entry), G^T on the vertex slices' entries
  scvs::Sell s2sell;
  scvs::DBuf<int64_t> s2_goff;
  int64_t s2_gn = 0;
  scvs::DBuf<float> s2_G32, s2_Gt32;
  bool fp32_ready = false;
  uint64_t generation = 0;  // bumped whenever the operator changes (assembly, boundary conditions)
  // boundary conditions
  std::vector<int32_t> bc_tags, bc_kinds, traction_tags;
  scvs::DBuf<int32_t> dmask, dirnodes;
  scvs::DBuf<double> loads, lpdinv;
  // pressure Laplacian G_F^T diag(M)^-1 G_F (vertex rows) for the Schur block
  scvs::DBuf<int64_t> lp_ptr;
  scvs::DBuf<int32_t> lp_col;
  scvs::DBuf<double> lp_val;
  scvs::DBuf<float> lp_val32;  // FP32 copy for the mixed-precision Schur block
  int64_t nnzl = 0;
  int64_t ndir = 0;
  double lp_lmax = 0.0;
  bool bc_set = false, assembled = false;
  double rho = 0.0, mu = 0.0;
  // lumped (Windkessel) outlets: outlet o adds Z_o(w) b_o b_o^T to the momentum rows,
  // b_o = int M_A n over the outlet (the load vector of its traction tag)
  int nwk = 0;
  std::vector<double> wk_par;          // [nwk][3]: rp, c, rd
  scvs::DBuf<double> wk_dpar;          // device copy
  scvs::DBuf<int64_t> wk_qoff;         // [2*nwk+1]: outlet o's free entries, then its Dirichlet entries
  scvs::DBuf<int32_t> wk_qdof;         // velocity unknown d*A + c of each entry
  scvs::DBuf<double> wk_qb;            // b at that unknown
  int64_t wk_nrow = 0;                 // distinct free rows of all outlets
  scvs::DBuf<int64_t> wk_roff;         // [wk_nrow+1] -> (outlet, b) pairs of each row
  scvs::DBuf<int32_t> wk_rdof, wk_rout;
  scvs::DBuf<double> wk_rb;
  // aggregation multigrid of the velocity block and the pressure Laplacian
  std::unique_ptr<scvs::MgData> mg;
};

namespace scvs {

// ---- utilities (util.hip) ----
// Exclusive scan of counts[n] into out[n+1]; returns the total (synchronizes).
int64_t exclusive_scan(const int64_t* counts, int64_t* out, int64_t n, hipStream_t s);
// Exclusive scan of int32 counts.
int64_t exclusive_scan32(const int32_t* counts, int64_t* out, int64_t n, hipStream_t s);
// Adjacency lists: for items i in [0,nitems) with nper target ids each, build
// per-target sorted lists of item indices.
void build_adjacency(const int32_t* ids, int64_t nitems, int nper, int64_t ntarget,
                     DBuf<int64_t>& ptr, DBuf<int32_t>& list, hipStream_t s);
inline bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}
// Launch-error check that is legal while the stream is being captured into a
// graph (errors of captured launches surface at instantiation or launch).
inline void launch_check(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive) return;
  SCVS_HIP(hipGetLastError());
}
template <class T>
void download(T* host, const T* dev, size_t n, hipStream_t s) {
  if (n) SCVS_HIP(hipMemcpyAsync(host, dev, n * sizeof(T), hipMemcpyDeviceToHost, s));
  SCVS_HIP(hipStreamSynchronize(s));
}

// ---- mesh.hip ----
void mesh_build(scvs_mesh m, hipStream_t s);
void mesh_boundary(scvs_mesh m, hipStream_t s);
void mesh_precond_setup(scvs_mesh m, hipStream_t s);
// Lumped outlets on traction tags (tags already validated); n = 0 removes them.
void mesh_windkessel(scvs_mesh m, int n, const int32_t* tags, const double* rp, const double* c, const double* rd,
                     hipStream_t s);
constexpr int SCVS_WK_MAX = 64;  // lumped outlets per mesh

// ---- assemble.hip ----
void assemble_mesh(scvs_mesh m, hipStream_t s);
void probe_mfma(const double* a, const double* b, double* d, hipStream_t s);
// Grundmann-Moeller rule of degree 2s+1 on the n-simplex (barycentric points).
void gm_rule(int n, int s, std::vector<double>& bary, std::vector<double>& w);

void mesh_set_midside(scvs_mesh m, int64_t n, const int32_t* ev, const double* xyz, hipStream_t s);

// ---- spmv.hip ----
// A per-slot vector argument: the vector of slot k starts at p + k * st.
template <class T>
struct SV {
  T* p = nullptr;
  int64_t st = 0;
  __host__ __device__ T* at(int k) const { return p + (int64_t)k * st; }
};
using VArg = SV<double2>;   // complex double vectors
using VArg32 = SV<float2>;  // complex single vectors (mixed-precision solves)

// Conversions between the complex element types.
template <class T>
__host__ __device__ inline T cvt2(double2 v);
template <>
__host__ __device__ inline double2 cvt2<double2>(double2 v) { return v; }
template <>
__host__ __device__ inline float2 cvt2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
__host__ __device__ inline double2 to_d2(double2 v) { return v; }
__host__ __device__ inline double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
// The active systems of one launch.
struct Batch;
__host__ __device__ inline double schur_w(const Batch& b, int slot);
struct Batch {
  int nact = 0;
  const int* act = nullptr;       // device [nact] slot indices
  const double* omega = nullptr;  // device [slots] w per slot
  const double* lv = nullptr;     // device [slots] Chebyshev upper bound, velocity block
  const double* insc = nullptr;   // device [slots * insc_st] input scale (nullptr = 1)
  int insc_st = 0, insc_idx = 0;
  double pen = 0.0;  // penalty: continuity block -pen * Mp (lumped), pen = epsilon / mu
  double wsteady = 0.0;  // w of the Schur block's Laplacian term for steady (w = 0) systems
  bool no_lumped = false;  // leave out the lumped-outlet terms
};
// w in the Schur block mu Mp^-1 + j w rho L^-1 of a system: its own, or wsteady when it is 0
__host__ __device__ inline double schur_w(const Batch& b, int slot) {
  const double w = b.omega[slot];
  return w != 0.0 ? w : b.wsteady;
}
enum { SPMV_APPLY = 0, SPMV_RESID = 1, SPMV_RHS = 2 };
// y = A x (APPLY), y = f - A x (RESID), y = [-sum P n - A x ; x on Dirichlet rows ; -G^T x] (RHS).
void spmv_full(scvs_mesh m, const Batch& b, VArg x, VArg y, int mode, bool maskcol, VArg f,
               const double2* trac, hipStream_t s);
// Block upper-triangular preconditioner z = P^-1 (insc * v); temps per slot.
struct PrecondArgs {
  int kv = 10, kp = 10;
  double ratio = 30.0;    // velocity block interval lmax/ratio..lmax
  double ratio_p = 30.0;  // pressure Laplacian interval
  int mixed = 0;  // 1: velocity block in FP32 (vt32, output z32); pressure block stays FP64
  VArg32 vt32;    // FP32 velocity temps: 4 * d*n2 per slot
  VArg32 z32;     // FP32 preconditioned vector (velocity part, plus a copy of the pressure part)
  VArg vt;  // velocity temps: 4 * d*n2 per slot (b, three rotating iterates)
  VArg pt;  // pressure temps: 4*nv per slot (r, d0, d1, x); 5*nv with pressure multigrid
  // multigrid blocks (vt/vt32 then hold 5*d*n2 per slot: level 0 of the velocity cycle)
  int vmg = 0, pmg = 0;
  int mg_nu = 2;
  int mg_post0 = 0;  // post-smoothing steps on the velocity's level 0 (0: mg_nu)
  double mg_ratio = 10.0;
  MgBufs mg;
};
// With zil (a buffer of nact*ndof values, FP32 in mixed mode) the result is written
// interleaved for spmv_apply_il instead of into z (z still receives the FP64 pressure
// part in the Schur step).
void precond_apply(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s,
                   void* zil = nullptr);
// Same, reading an FP32 input vector (FP32 Krylov basis).
void precond_apply(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg32 v, VArg z, hipStream_t s,
                   void* zil = nullptr);
// y = A x with x in the interleaved layout written by precond_apply(..., zil), into an
// FP64 or an FP32 output.
void spmv_apply_il(scvs_mesh m, const Batch& b, const void* xil, bool fp32, VArg y, hipStream_t s);
void spmv_apply_il(scvs_mesh m, const Batch& b, const void* xil, bool fp32, VArg32 y, hipStream_t s);
// y = f - A x (masked columns, as SPMV_RESID) with an FP32 output.
// tmp: an FP64 vector per slot, used (when lumped outlets are present) to form the
// residual in FP64 before it is rounded.
void spmv_resid32(scvs_mesh m, const Batch& b, VArg x, VArg32 y, VArg f, hipStream_t s, VArg tmp = VArg{});
// y = A x with FP32 matrix copies, FP32 input and FP32 accumulation; FP64 output.
void spmv_apply32(scvs_mesh m, const Batch& b, VArg32 x, VArg y, hipStream_t s);
// FP32 copies of the matrix values for mixed-precision solves (made once per assembly).
void make_fp32_copies(scvs_mesh m, hipStream_t s);
// Gershgorin bound of diag^-1 (mu Ks + |w| rho M) on the free rows, per slot.
void velocity_bounds(scvs_mesh m, const Batch& b, double* lv_out, hipStream_t s);

// ---- mg.hip ----
void mg_setup(scvs_mesh m, hipStream_t s);
// Bytes of the temporaries below level 0 for `slots` systems (complex elements of esize bytes).
size_t mg_buffer_bytes(scvs_mesh m, int slots, size_t esize, bool vel, bool pres);
void mg_assign(scvs_mesh m, int slots, size_t esize, bool vel, bool pres, char* base, void* vel0, void* pres0,
               double* vlam, MgBufs& out);
int mg_levels(scvs_mesh m, bool vel);
// Level-0 values in sliced rows for the cycle's precision (FP32 when f32).
void mg_sell_values(scvs_mesh m, bool f32, bool vel, bool pres, hipStream_t s);
// Sliced rows of an n-row CSR pattern (host row pointers, device pointers and columns);
// rows below `split` fill the first slices.
void sell_build(Sell& S, const std::vector<int64_t>& ptr, int64_t n, int64_t split, const int64_t* dptr,
                const int32_t* dcol, hipStream_t s);
// Sliced values from CSR values of the pattern the layout was built from.
template <class R>
void sell_values(const Sell& S, const int64_t* dptr, const R* a, DBuf<R>& out, hipStream_t s);
// The mesh's S2 in sliced rows with FP32 values (Ks, M, G, G^T; f32) and FP64 values
// (Ks, M; f64), each made once per assembly; needs the FP32 copies for f32.
void s2sell_setup(scvs_mesh m, bool f32, bool f64, hipStream_t s);
void s2sell_release_values(scvs_mesh m);
// Per system: smoother bounds of every velocity level and the coarsest level's dense inverse.
void mg_prepare(scvs_mesh m, const Batch& b, double* lam, int slots, double2* inv, float2* inv32, hipStream_t s);
int64_t mg_coarse_rows(scvs_mesh m);
// Levels of a hierarchy (0 velocity, 1 pressure; built if needed): rows, nonzeros and the
// nonzeros of the transfer to the next level, for up to maxlev levels; returns the count.
int mg_info(scvs_mesh m, int which, int maxlev, int64_t* rows, int64_t* nnz, int64_t* pnnz);
// Velocity V-cycle from the level-0 right-hand side and first iterate (k_vinit); the
// result goes to zil (interleaved) or, without it, to z (FP32 z32 in mixed mode).
void mg_velocity(scvs_mesh m, const Batch& b, const PrecondArgs& pa, void* zil, VArg z, hipStream_t s);
// Pressure-Laplacian V-cycle from the level-0 right-hand side and first iterate
// (k_pinit) and the FP64 Schur combination into z for the systems with w != 0.
void mg_pressure(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg v, VArg z, hipStream_t s);
void mg_pressure(scvs_mesh m, const Batch& b, const PrecondArgs& pa, VArg32 v, VArg z, hipStream_t s);

// ---- krylov.hip ----
int solve_systems(scvs_mesh m, int64_t nsys, const double* omega, const double* traction,
                  const void* g, const void* x0, void* u_out, void* p_out,
                  const scvs_solve_opts* o, scvs_report* rep);
void rhs_systems(scvs_mesh m, int64_t nsys, const double* omega, const double* traction,
                 const void* g, void* f);
// x[slot act[k]] = Dirichlet data g[k] on the Dirichlet nodes, zero elsewhere (walls too).
void scatter_dirichlet(scvs_mesh m, int64_t nsys, const void* g, VArg x, const int* act, hipStream_t s);

// ---- modes.hip ----
// Per system: squared L2(Gamma) norms of the traction data (hn2) and of the
// Dirichlet data on the Dirichlet facets (gn2); host outputs.
void boundary_norms(scvs_mesh m, int64_t nsys, const double* traction, const void* g, double* hn2, double* gn2);
// Per system: u^H (I_d (x) M) u and p^H Mp p (lumped pressure mass); host outputs.
void mode_norms(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2);
// The same with the partial sums in the library's file-scope device array (no allocation);
// noalloc_init resolves that array's address on the current device (called per context).
void mode_norms_noalloc(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2);
void noalloc_init(int device);

// ---- learned.hip ----
struct Mlp;
void herm_eig(int n, std::vector<std::complex<double>>& A, std::vector<double>& w,
              std::vector<std::complex<double>>& V);
void ws_build(scvs_ws w, int64_t S, const double* omega, const double2* snaps, int r, int width, int layers,
              uint64_t seed);
double ws_train(scvs_ws w, int epochs, double lr);
void ws_predict(scvs_ws w, int64_t n, const double* omega, const double* amp, double2* x0);
void ws_refine(scvs_ws w, int64_t n, const double* omega, const double* traction, const void* g, double2* x0);
double ws_loss_grad(scvs_ws w, int n, const float* x_host, const float* t_host, float* grads_host);
void probe_mfma_bf16(const float* a, const float* b, float* d, hipStream_t s);

// ---- synth.hip ----
void synthesize(hipStream_t s, int64_t nk, const double* omega, const double2* modes,
                int64_t nvals, int64_t nt, const double* times, double* out);

}  // namespace scvs


namespace scvs {
// ---- MLP object (device) ----
struct Mlp {
  std::vector<int> sizes;  // layer widths, sizes[0] = inputs
  int64_t nparam = 0;
  std::vector<int64_t> woff, boff;  // offsets of W_l and b_l in the flat parameter vector
  DBuf<float> p, g, m, v;           // parameters, gradients, Adam moments
  int64_t step = 0;
  void init(const std::vector<int>& sz, uint64_t seed, hipStream_t s) {
    sizes = sz;
    nparam = 0;
    woff.clear();
    boff.clear();
    for (size_t l = 0; l + 1 < sizes.size(); ++l) {
      woff.push_back(nparam);
      nparam += (int64_t)sizes[l] * sizes[l + 1];
      boff.push_back(nparam);
      nparam += sizes[l + 1];
    }
    std::vector<float> h(nparam, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    for (size_t l = 0; l + 1 < sizes.size(); ++l) {
      const float sc = 1.f / std::sqrt((float)sizes[l]);
      for (int64_t k = 0; k < (int64_t)sizes[l] * sizes[l + 1]; ++k) h[woff[l] + k] = sc * nd(rng);
    }
    p.upload(h.data(), nparam, s);
    g.alloc(nparam);
    m.alloc(nparam);
    v.alloc(nparam);
    m.zero(s);
    v.zero(s);
    step = 0;
  }
  int layers() const { return (int)sizes.size() - 1; }
};

// Forward pass for n samples; acts holds per layer the input H_l ([n][sizes[l]])
// and pre-activation Z_l ([n][sizes[l+1]]); returns the output pointer.
struct MlpWork {
  std::vector<DBuf<float>> H, Z, dH;
  DBuf<float> dZ;
  DBuf<double> part;
  int n = 0;
  void ensure(const Mlp& net, int nn) {
    if (nn <= n && !H.empty()) return;
    n = nn;
    const int L = net.layers();
    H.clear();
    Z.clear();
    dH.clear();
    H.resize(L + 1);
    Z.resize(L);
    dH.resize(L + 1);
    int mx = 0;
    for (int l = 0; l <= L; ++l) {
      H[l].alloc((size_t)n * net.sizes[l]);
      dH[l].alloc((size_t)n * net.sizes[l]);
      mx = std::max(mx, net.sizes[l]);
    }
    for (int l = 0; l < L; ++l) Z[l].alloc((size_t)n * net.sizes[l + 1]);
    dZ.alloc((size_t)n * mx);
    part.alloc(256);
  }
};

}  // namespace scvs

// ---- warm-start model ----
struct scvs_ws_s {
  scvs_mesh mesh = nullptr;
  int S = 0, r = 0;
  int64_t ndof = 0;
  double wmax = 1.0;
  double sigma0 = 0.0;            // largest singular value (scale of the targets)
  scvs::DBuf<double2> basis;      // [r][ndof]
  scvs::DBuf<double> sigma_d;     // [r]
  std::vector<double> sigma;      // [r]
  std::vector<double> omega;      // [S] snapshot frequencies
  std::vector<float> targets;     // [S][2r] standardized POD coefficients (t - tmean) / tscale
  std::vector<double> tmean, tscale;  // [2r] per output, over the snapshots
  scvs::DBuf<double> tstd_d;      // [4r] tmean then tscale on the device
  scvs::Mlp net;
  scvs::MlpWork work;
  scvs::DBuf<float> X, T;         // training inputs/targets on the device
  // reduced operator for the subspace correction: Q = [Q0; Q1; B] ([2r+nb][ndof]) with
  // A(w) phi_i = Q0_i + j w Q1_i + sum_o Z_o(w) Cb[o][i] B_o on unconstrained rows
  // (B_o the load vector of lumped outlet o, Cb = B^T Phi), and its Gram matrix H (host)
  uint64_t red_gen = ~0ull;
  int nb = 0;
  scvs::DBuf<double2> Q;
  std::vector<std::complex<double>> H, Cb;
};


// ---- device helpers ----
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

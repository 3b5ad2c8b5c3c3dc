// C ABI of the SCVS library: validation, object lifetime, error reporting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include <atomic>

#include "internal.hpp"

using scvs::DBuf;
using scvs::Error;
using scvs::fail;

namespace {

thread_local std::string g_last_error;

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return SCVS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SCVS_E_NOMEM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return SCVS_E_INVALID;
  }
}

void use_device(scvs_ctx c) { SCVS_HIP(hipSetDevice(c->device)); }

void require_ready(scvs_mesh m) {
  SCVS_REQUIRE(m, SCVS_E_INVALID, "mesh is null");
  SCVS_REQUIRE(m->bc_set, SCVS_E_STATE, "boundary conditions not set (call scvs_mesh_set_bc)");
  SCVS_REQUIRE(m->assembled, SCVS_E_STATE, "matrices not assembled (call scvs_assemble)");
}

// Options from the caller (or the defaults), validated.
scvs_solve_opts checked_opts(const scvs_solve_opts* opts) {
  scvs_solve_opts o;
  if (opts)
    o = *opts;
  else
    scvs_solve_opts_default(&o);
  SCVS_REQUIRE(o.rtol > 0.0 && o.restart >= 1 && o.restart <= SCVS_MMAX && o.max_iters >= 1 && o.cheb_vel >= 1 &&
                   o.cheb_pres >= 0 && o.cheb_ratio > 1.0 && o.max_batch >= 0 &&
                   (o.precision >= 0 && o.precision <= 2) && (o.orth == 0 || o.orth == 1) &&
                   (o.precision != 2 || o.orth == 1) && o.inner_rtol >= 0.0 && o.inner_rtol < 1.0 &&
                   (o.cheb_ratio_pres == 0.0 || o.cheb_ratio_pres > 1.0) && o.penalty >= 0.0 &&
                   std::isfinite(o.penalty) && (o.vel_block == 0 || o.vel_block == 1) &&
                   (o.pres_block == 0 || o.pres_block == 1) && o.mg_smooth >= 1 && o.mg_smooth <= 16 &&
                   o.mg_ratio > 1.0 && std::isfinite(o.mg_ratio) && o.steady_schur_omega >= 0.0 &&
                   std::isfinite(o.steady_schur_omega) && o.mg_post0 >= 0 && o.mg_post0 <= 16,
               SCVS_E_INVALID, "bad solve options");
  return o;
}

// Every option the autotuner does not choose (and that changes the solve), as a key.
std::string untuned_key(const scvs_solve_opts& oin) {
  scvs_solve_opts o = oin;
  o.restart = 0;
  if (o.vel_block == 1) {  // tuned with the multigrid velocity block
    o.mg_smooth = 0;
    o.mg_ratio = 0.0;
  } else {  // tuned with the Chebyshev velocity block
    o.cheb_vel = 0;
    o.cheb_pres = 0;
  }
  char buf[512];
  snprintf(buf, sizeof buf, "%.17g|%d|%.17g|%d|%d|%d|%d|%.17g|%.17g|%.17g|%d|%d|%d|%.17g|%.17g|%d|%d|%d", o.rtol,
           o.max_iters, o.cheb_ratio, o.max_batch, o.use_graph, o.precision, o.orth, o.cheb_ratio_pres, o.penalty,
           o.inner_rtol, o.vel_block, o.pres_block, o.mg_smooth, o.mg_ratio, o.steady_schur_omega, o.mg_post0,
           o.cheb_vel, o.cheb_pres);
  return buf;
}

}  // namespace

extern "C" {

const char* scvs_last_error(void) { return g_last_error.c_str(); }

const char* scvs_version(void) { return "scvs-gfx950 0.1"; }

int scvs_ctx_create(int device, void* stream, scvs_ctx* out) {
  return guarded([&] {
    SCVS_REQUIRE(out, SCVS_E_INVALID, "out is null");
    int n = 0;
    SCVS_HIP(hipGetDeviceCount(&n));
    SCVS_REQUIRE(device >= 0 && device < n, SCVS_E_INVALID, "device index out of range");
    SCVS_HIP(hipSetDevice(device));
    scvs::noalloc_init(device);
    auto* c = new scvs_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)stream;
    // The legacy null stream cannot be captured; graphs are recorded on a
    // private stream (nothing executes during capture) and launched on c->stream.
    if (hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      fail(SCVS_E_HIP, "hipStreamCreateWithFlags failed");
    }
    *out = c;
  });
}

int scvs_ctx_set_mem_cap(scvs_ctx ctx, uint64_t bytes) {
  return guarded([&] {
    SCVS_REQUIRE(ctx, SCVS_E_INVALID, "ctx is null");
    ctx->mem_cap = bytes;
  });
}

int scvs_ctx_destroy(scvs_ctx ctx) {
  return guarded([&] {
    if (ctx && ctx->capture) (void)hipStreamDestroy(ctx->capture);
    delete ctx;
  });
}

int scvs_mesh_create(scvs_ctx ctx, int dim, int64_t nv, const double* xyz, int64_t nc, const int32_t* cells,
                     int64_t nf, const int32_t* bfaces, const int32_t* btags, scvs_mesh* out) {
  return guarded([&] {
    SCVS_REQUIRE(ctx && out, SCVS_E_INVALID, "ctx or out is null");
    SCVS_REQUIRE(dim == 2 || dim == 3, SCVS_E_INVALID, "dim must be 2 or 3");
    SCVS_REQUIRE(nv > 0 && nc > 0 && nf >= 0, SCVS_E_INVALID, "counts must be positive (nf >= 0)");
    SCVS_REQUIRE(nv < INT32_MAX && nc < INT32_MAX, SCVS_E_INVALID, "counts exceed 32-bit indices");
    SCVS_REQUIRE(xyz && cells, SCVS_E_INVALID, "xyz or cells is null");
    SCVS_REQUIRE(nf == 0 || (bfaces && btags), SCVS_E_INVALID, "bfaces or btags is null");
    const int nvl = dim + 1;
    for (int64_t i = 0; i < nv * dim; ++i)
      SCVS_REQUIRE(std::isfinite(xyz[i]), SCVS_E_MESH, "non-finite vertex coordinate");
    for (int64_t c = 0; c < nc; ++c) {
      const int32_t* v = cells + c * nvl;
      for (int k = 0; k < nvl; ++k) {
        SCVS_REQUIRE(v[k] >= 0 && v[k] < nv, SCVS_E_MESH, "cell vertex index out of range");
        for (int l = 0; l < k; ++l) SCVS_REQUIRE(v[k] != v[l], SCVS_E_MESH, "cell repeats a vertex");
      }
      double J[3][3] = {};
      for (int r = 0; r < dim; ++r)
        for (int k = 0; k < dim; ++k) J[r][k] = xyz[(int64_t)v[k + 1] * dim + r] - xyz[(int64_t)v[0] * dim + r];
      double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                            : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                  J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                  J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      SCVS_REQUIRE(det != 0.0, SCVS_E_MESH, "degenerate cell (zero volume)");
    }
    for (int64_t i = 0; i < nf * dim; ++i)
      SCVS_REQUIRE(bfaces[i] >= 0 && bfaces[i] < nv, SCVS_E_MESH, "facet vertex index out of range");
    for (int64_t i = 0; i < nf; ++i) SCVS_REQUIRE(btags[i] >= 0, SCVS_E_INVALID, "negative facet tag");
    use_device(ctx);
    hipStream_t s = ctx->stream;
    auto m = std::make_unique<scvs_mesh_s>();
    m->ctx = ctx;
    static std::atomic<uint64_t> next_uid{1};
    m->uid = next_uid++;
    m->dim = dim;
    m->nvl = nvl;
    m->nn = nvl * (nvl + 1) / 2;
    m->nv = nv;
    m->nc = nc;
    m->nf = nf;
    m->xyz.upload(xyz, nv * dim, s);
    m->cells.upload(cells, nc * nvl, s);
    m->bfaces.upload(bfaces, nf * dim, s);
    m->btags.upload(btags, nf, s);
    scvs::mesh_build(m.get(), s);
    SCVS_REQUIRE(m->n2 < INT32_MAX, SCVS_E_CAPACITY, "more than 2^31 quadratic nodes");
    *out = m.release();
  });
}

int scvs_mesh_destroy(scvs_mesh mesh) {
  return guarded([&] {
    if (mesh) {
      use_device(mesh->ctx);
      SCVS_HIP(hipStreamSynchronize(mesh->ctx->stream));
      auto& t = mesh->ctx->tuned;
      for (auto it = t.begin(); it != t.end();) it = std::get<0>(it->first) == mesh->uid ? t.erase(it) : std::next(it);
    }
    delete mesh;
  });
}

int scvs_mesh_info(scvs_mesh m, scvs_mesh_info_t* info) {
  return guarded([&] {
    SCVS_REQUIRE(m && info, SCVS_E_INVALID, "mesh or info is null");
    info->dim = m->dim;
    info->nv = m->nv;
    info->nc = m->nc;
    info->nf = m->nf;
    info->ne = m->ne;
    info->n2 = m->n2;
    info->ndof = m->dim * m->n2 + m->nv;
    info->nnz_s2 = m->nnz;
    info->nnz_c21 = m->nnz21;
    info->ndir = m->ndir;
    info->ntraction = (int32_t)m->traction_tags.size();
    info->assembled = m->assembled ? 1 : 0;
  });
}

int scvs_mesh_set_midside(scvs_mesh m, int64_t n, const int32_t* ev, const double* xyz) {
  return guarded([&] {
    SCVS_REQUIRE(m, SCVS_E_INVALID, "mesh is null");
    SCVS_REQUIRE(n >= 0 && (n == 0 || (ev && xyz)), SCVS_E_INVALID, "bad midside arguments");
    for (int64_t i = 0; i < 2 * n; ++i)
      SCVS_REQUIRE(ev[i] >= 0 && ev[i] < m->nv, SCVS_E_INVALID, "midside edge vertex out of range");
    for (int64_t i = 0; i < n * m->dim; ++i)
      SCVS_REQUIRE(std::isfinite(xyz[i]), SCVS_E_INVALID, "non-finite midside coordinate");
    if (n == 0) return;
    use_device(m->ctx);
    scvs::mesh_set_midside(m, n, ev, xyz, m->ctx->stream);
    m->assembled = false;
    // the traction loads and lumped-outlet vectors were integrated on the old facets:
    // boundary conditions must be set again
    if (m->bc_set) scvs::mesh_windkessel(m, 0, nullptr, nullptr, nullptr, nullptr, m->ctx->stream);
    m->bc_set = false;
    m->generation++;
  });
}

int scvs_mesh_set_bc(scvs_mesh m, int n, const int32_t* tags, const int32_t* kinds) {
  return guarded([&] {
    SCVS_REQUIRE(m, SCVS_E_INVALID, "mesh is null");
    SCVS_REQUIRE(n >= 0 && (n == 0 || (tags && kinds)), SCVS_E_INVALID, "bad boundary-condition arguments");
    for (int i = 0; i < n; ++i) {
      SCVS_REQUIRE(kinds[i] >= SCVS_BC_FREE && kinds[i] <= SCVS_BC_TRACTION, SCVS_E_INVALID,
                   "unknown boundary-condition kind");
      for (int k = 0; k < i; ++k) SCVS_REQUIRE(tags[k] != tags[i], SCVS_E_INVALID, "tag listed twice");
    }
    use_device(m->ctx);
    m->bc_tags.assign(tags, tags + n);
    m->bc_kinds.assign(kinds, kinds + n);
    scvs::mesh_windkessel(m, 0, nullptr, nullptr, nullptr, nullptr, m->ctx->stream);
    scvs::mesh_boundary(m, m->ctx->stream);
    m->generation++;
    if (m->assembled) scvs::mesh_precond_setup(m, m->ctx->stream);
  });
}

int scvs_mesh_set_windkessel(scvs_mesh m, int n, const int32_t* tags, const double* rp, const double* c,
                             const double* rd) {
  return guarded([&] {
    SCVS_REQUIRE(m, SCVS_E_INVALID, "mesh is null");
    SCVS_REQUIRE(m->bc_set, SCVS_E_STATE, "boundary conditions not set (call scvs_mesh_set_bc)");
    SCVS_REQUIRE(n >= 0 && n <= scvs::SCVS_WK_MAX && (n == 0 || (tags && rp && c && rd)), SCVS_E_INVALID,
                 "bad lumped-outlet arguments");
    for (int i = 0; i < n; ++i) {
      SCVS_REQUIRE(std::find(m->traction_tags.begin(), m->traction_tags.end(), tags[i]) != m->traction_tags.end(),
                   SCVS_E_INVALID, "a lumped outlet must be a TRACTION tag");
      for (int k = 0; k < i; ++k) SCVS_REQUIRE(tags[k] != tags[i], SCVS_E_INVALID, "tag listed twice");
      SCVS_REQUIRE(std::isfinite(rp[i]) && std::isfinite(c[i]) && std::isfinite(rd[i]) && rp[i] >= 0.0 &&
                       c[i] >= 0.0 && rd[i] >= 0.0,
                   SCVS_E_INVALID, "Windkessel parameters must be finite and >= 0");
    }
    use_device(m->ctx);
    scvs::mesh_windkessel(m, n, tags, rp, c, rd, m->ctx->stream);
    m->generation++;
  });
}

int scvs_assemble(scvs_mesh m, double rho, double mu) {
  return guarded([&] {
    SCVS_REQUIRE(m, SCVS_E_INVALID, "mesh is null");
    SCVS_REQUIRE(rho > 0.0 && mu > 0.0 && std::isfinite(rho) && std::isfinite(mu), SCVS_E_INVALID,
                 "rho and mu must be positive and finite");
    use_device(m->ctx);
    scvs::assemble_mesh(m, m->ctx->stream);
    m->rho = rho;
    m->mu = mu;
    m->assembled = true;
    m->fp32_ready = false;
    scvs::s2sell_release_values(m);
    m->generation++;
    if (m->bc_set) scvs::mesh_precond_setup(m, m->ctx->stream);
  });
}

int scvs_mesh_export(scvs_mesh m, int which, void* out) {
  return guarded([&] {
    SCVS_REQUIRE(m && out, SCVS_E_INVALID, "mesh or out is null");
    use_device(m->ctx);
    hipStream_t s = m->ctx->stream;
    const int D = m->dim;
    auto need_asm = [&] { SCVS_REQUIRE(m->assembled, SCVS_E_STATE, "matrices not assembled"); };
    auto need_bc = [&] { SCVS_REQUIRE(m->bc_set, SCVS_E_STATE, "boundary conditions not set"); };
    switch (which) {
      case SCVS_X_EDGES: scvs::download((int32_t*)out, m->edges.p, 2 * m->ne, s); break;
      case SCVS_X_C2N: scvs::download((int32_t*)out, m->c2n.p, m->nc * m->nn, s); break;
      case SCVS_X_ROWPTR: scvs::download((int64_t*)out, m->rowptr.p, m->n2 + 1, s); break;
      case SCVS_X_COL: scvs::download((int32_t*)out, m->col.p, m->nnz, s); break;
      case SCVS_X_KS: need_asm(); scvs::download((double*)out, m->Ks.p, m->nnz, s); break;
      case SCVS_X_M: need_asm(); scvs::download((double*)out, m->M.p, m->nnz, s); break;
      case SCVS_X_G: need_asm(); scvs::download((double*)out, m->G.p, D * m->nnz21, s); break;
      case SCVS_X_MP: need_asm(); scvs::download((double*)out, m->Mp.p, m->nv, s); break;
      case SCVS_X_DIRNODES: need_bc(); scvs::download((int32_t*)out, m->dirnodes.p, m->ndir, s); break;
      case SCVS_X_DMASK: need_bc(); scvs::download((int32_t*)out, m->dmask.p, m->n2, s); break;
      case SCVS_X_LOADS:
        need_bc();
        scvs::download((double*)out, m->loads.p, m->traction_tags.size() * m->n2 * D, s);
        break;
      case SCVS_X_NODEXYZ: {
        std::vector<double> h(m->nv * D), e(m->ne * D);
        scvs::download(h.data(), m->xyz.p, h.size(), s);
        scvs::download(e.data(), m->exyz.p, e.size(), s);
        memcpy(out, h.data(), h.size() * sizeof(double));
        memcpy((double*)out + h.size(), e.data(), e.size() * sizeof(double));
        break;
      }
      case SCVS_X_C21PTR: scvs::download((int64_t*)out, m->rowptr21.p, m->n2 + 1, s); break;
      case SCVS_X_C21COL: {
        // C21 is stored as the vertex-column prefix of each S2 row
        std::vector<int64_t> rp(m->n2 + 1);
        std::vector<int32_t> col(m->nnz), nvc(m->n2);
        scvs::download(rp.data(), m->rowptr.p, m->n2 + 1, s);
        scvs::download(col.data(), m->col.p, m->nnz, s);
        scvs::download(nvc.data(), m->nvc.p, m->n2, s);
        int32_t* o = (int32_t*)out;
        for (int64_t a = 0; a < m->n2; ++a)
          for (int32_t k = 0; k < nvc[a]; ++k) *o++ = col[rp[a] + k];
        break;
      }
      default: fail(SCVS_E_INVALID, "unknown export selector");
    }
  });
}

int scvs_spmv(scvs_mesh m, int64_t nsys, const double* omega, const void* x, void* y) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && omega && x && y, SCVS_E_INVALID, "bad spmv arguments");
    SCVS_REQUIRE(nsys <= 4096, SCVS_E_INVALID, "at most 4096 systems per call");
    for (int64_t k = 0; k < nsys; ++k) SCVS_REQUIRE(std::isfinite(omega[k]), SCVS_E_INVALID, "non-finite omega");
    use_device(m->ctx);
    hipStream_t s = m->ctx->stream;
    const int64_t ndof = m->dim * m->n2 + m->nv;
    DBuf<double> om;
    DBuf<int> act;
    std::vector<int> a(nsys);
    for (int64_t k = 0; k < nsys; ++k) a[k] = (int)k;
    om.upload(omega, nsys, s);
    act.upload(a.data(), nsys, s);
    scvs::Batch b;
    b.nact = (int)nsys;
    b.act = act;
    b.omega = om;
    scvs::spmv_full(m, b, scvs::VArg{(double2*)x, ndof}, scvs::VArg{(double2*)y, ndof}, scvs::SPMV_APPLY, true,
                    scvs::VArg{}, nullptr, s);
    SCVS_HIP(hipStreamSynchronize(s));
  });
}

int scvs_rhs(scvs_mesh m, int64_t nsys, const double* omega, const double* traction, const void* g, void* f) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && nsys <= 4096 && omega && f, SCVS_E_INVALID, "bad rhs arguments");
    SCVS_REQUIRE(m->traction_tags.empty() || traction, SCVS_E_INVALID, "traction is null");
    SCVS_REQUIRE(m->ndir == 0 || g, SCVS_E_INVALID, "g is null but the mesh has Dirichlet nodes");
    use_device(m->ctx);
    scvs::rhs_systems(m, nsys, omega, traction, m->ndir ? g : nullptr, f);
  });
}

void scvs_solve_opts_default(scvs_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-10;
  o->restart = 200;
  o->max_iters = 20000;
  o->cheb_vel = 12;
  o->cheb_pres = 50;
  o->cheb_ratio = 300.0;
  o->max_batch = 0;
  o->use_graph = 1;
  o->verbose = 0;
  o->precision = 0;
  o->orth = 1;
  o->cheb_ratio_pres = 1000.0;
  o->penalty = 0.0;
  o->inner_rtol = 3e-5;
  o->vel_block = 0;
  o->pres_block = 0;
  o->mg_smooth = 2;
  o->mg_ratio = 4.0;
  o->steady_schur_omega = 0.0;
  o->mg_post0 = 0;
}

int scvs_solve(scvs_mesh m, int64_t nsys, const double* omega, const double* traction, const void* g,
               const void* x0, void* u_out, void* p_out, const scvs_solve_opts* opts, scvs_report* rep) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && omega && u_out && p_out, SCVS_E_INVALID, "bad solve arguments");
    SCVS_REQUIRE(m->traction_tags.empty() || traction, SCVS_E_INVALID, "traction is null");
    SCVS_REQUIRE(m->ndir == 0 || g, SCVS_E_INVALID, "g is null but the mesh has Dirichlet nodes");
    const scvs_solve_opts o = checked_opts(opts);
    for (int64_t k = 0; k < nsys; ++k) SCVS_REQUIRE(std::isfinite(omega[k]), SCVS_E_INVALID, "non-finite omega");
    use_device(m->ctx);
    scvs::solve_systems(m, nsys, omega, traction, m->ndir ? g : nullptr, x0, u_out, p_out, &o, rep);
  });
}

int scvs_solve_groups(int n, const scvs_solve_group* groups) {
  if (!(n >= 1 && n <= 64 && groups)) {
    g_last_error = "bad group arguments";
    return SCVS_E_INVALID;
  }
  for (int i = 0; i < n; ++i) {
    if (!groups[i].mesh) {
      g_last_error = "group mesh is null";
      return SCVS_E_INVALID;
    }
    for (int k = 0; k < i; ++k)
      if (groups[k].mesh->ctx == groups[i].mesh->ctx) {
        g_last_error = "groups must use distinct contexts (one stream each)";
        return SCVS_E_INVALID;
      }
  }
  std::vector<int> code(n, SCVS_OK);
  std::vector<std::string> msg(n);
  auto run = [&](int i) {
    const scvs_solve_group& gr = groups[i];
    code[i] = scvs_solve(gr.mesh, gr.nsys, gr.omega, gr.traction, gr.g, gr.x0, gr.u_out, gr.p_out, gr.opts, gr.rep);
    if (code[i] != SCVS_OK) msg[i] = g_last_error;  // this thread's message
  };
  std::vector<std::thread> th;
  for (int i = 1; i < n; ++i) th.emplace_back(run, i);
  run(0);
  for (auto& t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (code[i] != SCVS_OK) {
      g_last_error = "group " + std::to_string(i) + ": " + msg[i];
      return code[i];
    }
  g_last_error.clear();
  return SCVS_OK;
}

int scvs_autotune(scvs_mesh m, int64_t nsys, const double* omega, const double* traction, const void* g,
                  const scvs_solve_opts* base, scvs_solve_opts* best, double* best_ms) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && nsys <= 4096 && omega && best, SCVS_E_INVALID, "bad autotune arguments");
    SCVS_REQUIRE(m->traction_tags.empty() || traction, SCVS_E_INVALID, "traction is null");
    SCVS_REQUIRE(m->ndir == 0 || g, SCVS_E_INVALID, "g is null but the mesh has Dirichlet nodes");
    const scvs_solve_opts b = checked_opts(base);
    for (int64_t k = 0; k < nsys; ++k) SCVS_REQUIRE(std::isfinite(omega[k]), SCVS_E_INVALID, "non-finite omega");
    use_device(m->ctx);
    const auto key = std::make_tuple(m->uid, m->generation, nsys, untuned_key(b));
    auto hit = m->ctx->tuned.find(key);
    if (hit == m->ctx->tuned.end()) {
      scvs::DBuf<double2> u, p;
      u.alloc((size_t)nsys * m->n2 * m->dim);
      p.alloc((size_t)nsys * m->nv);
      std::vector<scvs_report> rep(nsys);
      scvs_ctx_s::Tuned pick{b.restart, b.cheb_vel, b.cheb_pres, b.mg_smooth, b.mg_ratio, -1.0};
      std::vector<scvs_solve_opts> cand;
      if (b.vel_block == 1) {
        for (int mm : {30, 40, 60})
          for (int sm : {1, 2})
            for (double rt : {4.0, 10.0}) {
              scvs_solve_opts c = b;
              c.restart = mm;
              c.mg_smooth = sm;
              c.mg_ratio = rt;
              cand.push_back(c);
            }
      } else {
        for (int mm : {160, 220})
          for (int kp : {30, 50})
            for (int kv : {10, 12}) {
              scvs_solve_opts c = b;
              c.restart = std::min(mm, SCVS_MMAX);
              c.cheb_pres = kp;
              c.cheb_vel = kv;
              cand.push_back(c);
            }
      }
      for (const scvs_solve_opts& c : cand) {
        const auto t0 = std::chrono::steady_clock::now();
        scvs::solve_systems(m, nsys, omega, traction, m->ndir ? g : nullptr, nullptr, u.p, p.p, &c, rep.data());
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        bool ok = true;
        for (const auto& r : rep) ok = ok && r.status == 0;
        if (b.verbose)
          fprintf(stderr, "[scvs] autotune m %d Chebyshev %d/%d multigrid %d steps ratio %g: %.1f ms%s\n", c.restart,
                  c.cheb_vel, c.cheb_pres, c.mg_smooth, c.mg_ratio, ms, ok ? "" : " (not converged)");
        if (ok && (pick.ms < 0.0 || ms < pick.ms)) pick = {c.restart, c.cheb_vel, c.cheb_pres, c.mg_smooth, c.mg_ratio, ms};
      }
      SCVS_REQUIRE(pick.ms >= 0.0, SCVS_E_STATE, "no candidate configuration converged");
      hit = m->ctx->tuned.emplace(key, pick).first;
    }
    // the tuned fields over the caller's own options
    *best = b;
    best->restart = hit->second.restart;
    best->cheb_vel = hit->second.cheb_vel;
    best->cheb_pres = hit->second.cheb_pres;
    best->mg_smooth = hit->second.mg_smooth;
    best->mg_ratio = hit->second.mg_ratio;
    if (best_ms) *best_ms = hit->second.ms;
  });
}

int scvs_boundary_norms(scvs_mesh m, int64_t nsys, const double* traction, const void* g, double* hn2,
                        double* gn2) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && nsys <= 4096 && hn2 && gn2, SCVS_E_INVALID, "bad boundary-norm arguments");
    SCVS_REQUIRE(m->traction_tags.empty() || traction, SCVS_E_INVALID, "traction is null");
    SCVS_REQUIRE(m->ndir == 0 || g, SCVS_E_INVALID, "g is null but the mesh has Dirichlet nodes");
    use_device(m->ctx);
    scvs::boundary_norms(m, nsys, traction, m->ndir ? g : nullptr, hn2, gn2);
  });
}

int scvs_mode_norms(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && nsys <= 65535 && u && p && un2 && pn2, SCVS_E_INVALID, "bad mode-norm arguments");
    use_device(m->ctx);
    scvs::mode_norms(m, nsys, u, p, un2, pn2);
  });
}

int scvs_mode_norms_noalloc(scvs_mesh m, int64_t nsys, const void* u, const void* p, double* un2, double* pn2) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE(nsys > 0 && u && p && un2 && pn2, SCVS_E_INVALID, "bad mode-norm arguments");
    use_device(m->ctx);
    scvs::mode_norms_noalloc(m, nsys, u, p, un2, pn2);
  });
}

int scvs_mesh_mg_info(scvs_mesh m, int which, int maxlev, int64_t* rows, int64_t* nnz, int64_t* pnnz,
                      int* nlev) {
  return guarded([&] {
    require_ready(m);
    SCVS_REQUIRE((which == 0 || which == 1) && maxlev >= 0 && (maxlev == 0 || (rows && nnz && pnnz)) && nlev,
                 SCVS_E_INVALID, "bad multigrid-info arguments");
    use_device(m->ctx);
    *nlev = scvs::mg_info(m, which, maxlev, rows, nnz, pnnz);
  });
}

int scvs_select_modes(int64_t nk, const double* omega, const double* hn2, const double* gn2, double eps,
                      int consecutive, int64_t* order, int64_t* count, double* err) {
  return guarded([&] {
    SCVS_REQUIRE(nk > 0 && omega && hn2 && gn2 && order && count && eps >= 0.0, SCVS_E_INVALID,
                 "bad mode-selection arguments");
    // two-sided weights: the zeroth mode once, every other mode twice (Parseval)
    std::vector<double> w(nk);
    double H = 0.0, Gs = 0.0;
    for (int64_t k = 0; k < nk; ++k) {
      SCVS_REQUIRE(std::isfinite(omega[k]) && hn2[k] >= 0.0 && gn2[k] >= 0.0, SCVS_E_INVALID, "bad mode norms");
      w[k] = omega[k] == 0.0 ? 1.0 : 2.0;
      H += w[k] * hn2[k];
      Gs += w[k] * gn2[k];
    }
    auto share = [&](int64_t k) { return (H > 0.0 ? w[k] * hn2[k] / H : 0.0) + (Gs > 0.0 ? w[k] * gn2[k] / Gs : 0.0); };
    std::vector<int64_t> ord(nk);
    for (int64_t k = 0; k < nk; ++k) ord[k] = k;
    if (!consecutive)
      std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return share(a) > share(b); });
    // e_M^2 = (truncated traction energy) + (truncated Dirichlet energy), both relative;
    // tail[i] = sum of the shares of ord[i..nk), summed directly (no cancellation)
    std::vector<double> tail(nk + 1, 0.0);
    for (int64_t i = nk - 1; i >= 0; --i) tail[i] = tail[i + 1] + share(ord[i]);
    int64_t n = 1;  // at least one mode
    while (n < nk && !(tail[n] < eps * eps)) ++n;
    for (int64_t k = 0; k < nk; ++k) order[k] = ord[k];
    *count = n;
    if (err) *err = std::sqrt(tail[n]);
  });
}

int scvs_mode_increments(int64_t n, const double* omega, const double* un2, double* inc) {
  return guarded([&] {
    SCVS_REQUIRE(n > 0 && omega && un2 && inc, SCVS_E_INVALID, "bad increment arguments");
    double tot = 0.0;
    for (int64_t k = 0; k < n; ++k) {
      const double wk = (omega[k] == 0.0 ? 1.0 : 2.0) * un2[k];
      tot += wk;
      inc[k] = tot > 0.0 ? std::sqrt(wk / tot) : 0.0;
    }
  });
}

int scvs_synthesize(scvs_ctx ctx, int64_t nk, const double* omega, const void* modes, int64_t nvals, int64_t nt,
                    const double* times, void* out) {
  return guarded([&] {
    SCVS_REQUIRE(ctx && omega && (nt == 0 || times) && ((modes && out) || nt == 0 || nvals == 0), SCVS_E_INVALID,
                 "bad synthesis arguments");
    SCVS_REQUIRE(nk >= 1 && nk <= 256 && nvals >= 0 && nt >= 0, SCVS_E_INVALID, "bad synthesis sizes");
    for (int64_t k = 0; k < nk; ++k)
      SCVS_REQUIRE(std::isfinite(omega[k]) && omega[k] >= 0.0, SCVS_E_INVALID, "omega must be finite and >= 0");
    for (int64_t n = 0; n < nt; ++n) SCVS_REQUIRE(std::isfinite(times[n]), SCVS_E_INVALID, "non-finite time");
    use_device(ctx);
    scvs::synthesize(ctx->stream, nk, omega, (const double2*)modes, nvals, nt, times, (double*)out);
  });
}

int scvs_ws_create(scvs_mesh mesh, int64_t nsnap, const double* omega, const void* snaps, int rank, int width,
                   int layers, uint64_t seed, scvs_ws* out) {
  return guarded([&] {
    SCVS_REQUIRE(mesh && omega && snaps && out, SCVS_E_INVALID, "null warm-start argument");
    SCVS_REQUIRE(nsnap >= 1 && nsnap <= 128, SCVS_E_INVALID, "nsnap must be in 1..128");
    SCVS_REQUIRE(rank >= 1 && rank <= nsnap && rank <= 64, SCVS_E_INVALID, "rank must be in 1..min(nsnap, 64)");
    SCVS_REQUIRE(width >= 8 && width <= 1024 && layers >= 2 && layers <= 8, SCVS_E_INVALID, "bad MLP shape");
    for (int64_t k = 0; k < nsnap; ++k) SCVS_REQUIRE(std::isfinite(omega[k]), SCVS_E_INVALID, "non-finite omega");
    use_device(mesh->ctx);
    auto w = std::make_unique<scvs_ws_s>();
    w->mesh = mesh;
    w->ndof = mesh->dim * mesh->n2 + mesh->nv;
    scvs::ws_build(w.get(), nsnap, omega, (const double2*)snaps, rank, width, layers, seed);
    *out = w.release();
  });
}

int scvs_ws_train(scvs_ws ws, int epochs, double lr, double* loss) {
  return guarded([&] {
    SCVS_REQUIRE(ws && epochs >= 0 && lr > 0.0, SCVS_E_INVALID, "bad training arguments");
    use_device(ws->mesh->ctx);
    const double l = scvs::ws_train(ws, epochs, lr);
    if (loss) *loss = l;
  });
}

int scvs_ws_predict(scvs_ws ws, int64_t n, const double* omega, const double* amp, void* x0) {
  return guarded([&] {
    SCVS_REQUIRE(ws && n >= 1 && n <= 4096 && omega && amp && x0, SCVS_E_INVALID, "bad prediction arguments");
    use_device(ws->mesh->ctx);
    scvs::ws_predict(ws, n, omega, amp, (double2*)x0);
  });
}

int scvs_ws_refine(scvs_ws ws, int64_t n, const double* omega, const double* traction, const void* g, void* x0) {
  return guarded([&] {
    SCVS_REQUIRE(ws && n >= 1 && n <= 4096 && omega && x0, SCVS_E_INVALID, "bad refine arguments");
    scvs_mesh m = ws->mesh;
    require_ready(m);
    SCVS_REQUIRE(m->dim * m->n2 + m->nv == ws->ndof, SCVS_E_STATE, "mesh changed size since the model was built");
    SCVS_REQUIRE(m->traction_tags.empty() || traction, SCVS_E_INVALID, "traction is null");
    SCVS_REQUIRE(m->ndir == 0 || g, SCVS_E_INVALID, "g is null but the mesh has Dirichlet nodes");
    for (int64_t k = 0; k < n; ++k) SCVS_REQUIRE(std::isfinite(omega[k]), SCVS_E_INVALID, "non-finite omega");
    use_device(m->ctx);
    scvs::ws_refine(ws, n, omega, traction, m->ndir ? g : nullptr, (double2*)x0);
  });
}

int scvs_ws_destroy(scvs_ws ws) {
  return guarded([&] { delete ws; });
}

int scvs_ws_export(scvs_ws ws, int which, void* out) {
  return guarded([&] {
    SCVS_REQUIRE(ws && out, SCVS_E_INVALID, "null argument");
    use_device(ws->mesh->ctx);
    hipStream_t s = ws->mesh->ctx->stream;
    switch (which) {
      case SCVS_WS_SIGMA: memcpy(out, ws->sigma.data(), sizeof(double) * ws->r); break;
      case SCVS_WS_BASIS:
        SCVS_HIP(hipMemcpyAsync(out, ws->basis.p, sizeof(double2) * ws->r * ws->ndof, hipMemcpyDeviceToDevice, s));
        SCVS_HIP(hipStreamSynchronize(s));
        break;
      case SCVS_WS_PARAMS: scvs::download((float*)out, ws->net.p.p, ws->net.nparam, s); break;
      case SCVS_WS_TARGETS: memcpy(out, ws->targets.data(), sizeof(float) * ws->targets.size()); break;
      case SCVS_WS_NPARAM: *(int64_t*)out = ws->net.nparam; break;
      case SCVS_WS_TMEAN: memcpy(out, ws->tmean.data(), sizeof(double) * ws->tmean.size()); break;
      case SCVS_WS_TSCALE: memcpy(out, ws->tscale.data(), sizeof(double) * ws->tscale.size()); break;
      default: fail(SCVS_E_INVALID, "unknown export selector");
    }
  });
}

int scvs_ws_set_params(scvs_ws ws, const float* params) {
  return guarded([&] {
    SCVS_REQUIRE(ws && params, SCVS_E_INVALID, "null argument");
    use_device(ws->mesh->ctx);
    hipStream_t s = ws->mesh->ctx->stream;
    SCVS_HIP(hipMemcpyAsync(ws->net.p.p, params, sizeof(float) * ws->net.nparam, hipMemcpyHostToDevice, s));
    SCVS_HIP(hipStreamSynchronize(s));
  });
}

int scvs_ws_loss_grad(scvs_ws ws, int64_t n, const float* x, const float* t, double* loss, float* grads) {
  return guarded([&] {
    SCVS_REQUIRE(ws && n >= 1 && n <= 65536 && x && t && loss && grads, SCVS_E_INVALID, "bad arguments");
    use_device(ws->mesh->ctx);
    *loss = scvs::ws_loss_grad(ws, (int)n, x, t, grads);
  });
}

int scvs_herm_eig(int n, const double* a, double* w, double* v) {
  return guarded([&] {
    SCVS_REQUIRE(n >= 1 && n <= 4096 && a && w && v, SCVS_E_INVALID, "bad eigen-decomposition arguments");
    std::vector<std::complex<double>> A((size_t)n * n), V;
    memcpy(A.data(), a, sizeof(double) * 2 * n * n);
    std::vector<double> ww;
    scvs::herm_eig(n, A, ww, V);
    memcpy(w, ww.data(), sizeof(double) * n);
    memcpy(v, V.data(), sizeof(double) * 2 * n * n);
  });
}

int scvs_probe_mfma_bf16(scvs_ctx ctx, const float* a, const float* b, float* d) {
  return guarded([&] {
    SCVS_REQUIRE(ctx && a && b && d, SCVS_E_INVALID, "null argument");
    use_device(ctx);
    scvs::probe_mfma_bf16(a, b, d, ctx->stream);
  });
}

int scvs_profile_enable(scvs_ctx ctx, int on) {
  return guarded([&] {
    SCVS_REQUIRE(ctx, SCVS_E_INVALID, "ctx is null");
    use_device(ctx);
    ctx->prof.resolve();
    ctx->prof.on = on != 0;
  });
}

int scvs_profile_read(scvs_ctx ctx, int max, scvs_kernel_stat* out, int* n) {
  return guarded([&] {
    SCVS_REQUIRE(ctx && n && max >= 0 && (max == 0 || out), SCVS_E_INVALID, "bad profile arguments");
    use_device(ctx);
    ctx->prof.resolve();
    int k = 0;
    for (auto& kv : ctx->prof.stats) {
      if (k >= max) break;
      scvs_kernel_stat& o = out[k++];
      memset(o.name, 0, sizeof(o.name));
      strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
      o.launches = kv.second.launches;
      o.total_ms = kv.second.ms;
      o.bytes = kv.second.bytes;
    }
    *n = k;
    ctx->prof.stats.clear();
  });
}

int scvs_probe_mfma(scvs_ctx ctx, const double* a, const double* b, double* d) {
  return guarded([&] {
    SCVS_REQUIRE(ctx && a && b && d, SCVS_E_INVALID, "null argument");
    use_device(ctx);
    scvs::probe_mfma(a, b, d, ctx->stream);
  });
}

}  // extern "C"

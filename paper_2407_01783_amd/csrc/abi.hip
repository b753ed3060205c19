// extern "C" entry points of libstokes (declared in include/stokes.h):
// argument validation (before any HIP call), batching of right-hand sides,
// conversion between the caller layout and the internal layout, and error
// reporting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>

#include "kernels.h"
#include "ops.h"
#include "solver.h"

// Device scratch of stokes_residual_noalloc: one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: kernels and copies take the per-device address that
// hipGetSymbolAddress returns (g_scratch_dev below).
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace stokes {

namespace {
thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current (the caller makes it current).
void* scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error(STOKES_ERR_UNSUPPORTED, "device index out of range for scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(STOKES_ERR_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}
}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void DevBuf::alloc(size_t b) {
  release();
  if (b == 0) b = 8;
  if (hipMalloc(&p, b) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error(STOKES_ERR_ALLOC, "hipMalloc of " + std::to_string(b) + " bytes failed");
  }
  bytes = b;
}

void DevBuf::ensure(size_t b) {
  if (b <= bytes && p) return;
  alloc(std::max(b, bytes + bytes / 4));
}

namespace {

int64_t ipow64(int64_t b, int e) { return ipow(b, e); }

stokes_status check_problem(const stokes_problem* p) {
  if (!p) throw Error(STOKES_ERR_ARG, "problem is NULL");
  if (p->dim != 2 && p->dim != 3) throw Error(STOKES_ERR_ARG, "dim must be 2 or 3");
  if (p->n < 1) throw Error(STOKES_ERR_ARG, "n must be >= 1");
  if (!(p->mu > 0) || !std::isfinite(p->mu)) throw Error(STOKES_ERR_ARG, "mu must be finite and > 0");
  if (!(p->alpha > 0) || !std::isfinite(p->alpha)) throw Error(STOKES_ERR_ARG, "alpha must be finite and > 0");
  if (!(p->gamma >= 0) || !std::isfinite(p->gamma)) throw Error(STOKES_ERR_ARG, "gamma must be finite and >= 0");
  if (!(p->jitter >= 0 && p->jitter <= 0.2)) throw Error(STOKES_ERR_ARG, "jitter must be in [0, 0.2]");
  if ((p->flags & ~(STOKES_FLAG_STRAIN | STOKES_FLAG_P3)) != 0)
    throw Error(STOKES_ERR_ARG, "flags must combine STOKES_FLAG_STRAIN and STOKES_FLAG_P3 only");
  const int order = (p->flags & STOKES_FLAG_P3) ? 3 : 2;
  const int64_t n2 = ipow64(order * int64_t(p->n) + 1, p->dim);
  if (n2 >= (int64_t(1) << 31) / 4) throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large for 32-bit indices");
  return STOKES_OK;
}

void check_opts(const stokes_solve_opts* o) {
  if (!o) throw Error(STOKES_ERR_ARG, "opts is NULL");
  if (o->precision != STOKES_FP64 && o->precision != STOKES_MIXED) throw Error(STOKES_ERR_ARG, "precision");
  if (!(o->rtol > 0 && o->rtol < 1)) throw Error(STOKES_ERR_ARG, "rtol must be in (0, 1)");
  if (o->max_outer < 1 || o->max_inner < 1 || o->max_refine < 0) throw Error(STOKES_ERR_ARG, "iteration caps");
  if (o->restart < 1 || o->restart > 63) throw Error(STOKES_ERR_ARG, "restart must be in [1, 63]");
  if (o->inner_mode != STOKES_INNER_TOL && o->inner_mode != STOKES_INNER_FIXED) throw Error(STOKES_ERR_ARG, "inner_mode");
  if (o->cheb_degree < 1 || o->cheb_degree > 16) throw Error(STOKES_ERR_ARG, "cheb_degree must be in [1, 16]");
  if (!(o->inner_rtol_u > 0 && o->inner_rtol_u < 1) || !(o->inner_rtol_p > 0 && o->inner_rtol_p < 1))
    throw Error(STOKES_ERR_ARG, "inner tolerances must be in (0, 1)");
  if (o->schur_pc < 0 || o->schur_pc > 2) throw Error(STOKES_ERR_ARG, "schur_pc");
  if (o->coupled_pc < 0 || o->coupled_pc > 2) throw Error(STOKES_ERR_ARG, "coupled_pc");
  if (o->inner_its_u < 0 || o->inner_its_u > 1000 || o->inner_its_p < 0 || o->inner_its_p > 1000)
    throw Error(STOKES_ERR_ARG, "inner_its_u / inner_its_p must be in [0, 1000]");
  if (o->vel_pc != STOKES_VEL_CHEB && o->vel_pc != STOKES_VEL_MG) throw Error(STOKES_ERR_ARG, "vel_pc");
  if (o->arnoldi_fp64 < 0 || o->arnoldi_fp64 > 2) throw Error(STOKES_ERR_ARG, "arnoldi_fp64 must be 0, 1 or 2");
  if (o->profile < 0 || o->profile > 2) throw Error(STOKES_ERR_ARG, "profile must be 0, 1 or 2");
}

template <class F>
stokes_status guard(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return STOKES_ERR_ALLOC;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return STOKES_ERR_STATE;
  }
}

void sizes_of(const HostMesh& m, const HostCsr* P2full, int64_t sizes[10]);

// velocity x velocity, pressure x velocity, pressure x pressure
void patterns(const HostMesh& m, HostCsr& P2full, HostCsr& Bfull, HostCsr& P1) {
  element_pattern(m.p2, m.nloc, m.n_p2, m.p2, m.nloc, m.n_p2, m.n_e, P2full);
  element_pattern(m.q, m.nqloc, m.n_q, m.p2, m.nloc, m.n_p2, m.n_e, Bfull);
  element_pattern(m.q, m.nqloc, m.n_q, m.q, m.nqloc, m.n_q, m.n_e, P1);
}

int order_of(const stokes_problem* p) { return (p->flags & STOKES_FLAG_P3) ? 3 : 2; }

std::vector<int32_t> interior_map(const HostMesh& m, int64_t& nI) {
  std::vector<int32_t> map(m.n_p2, -1);
  nI = 0;
  for (int64_t v = 0; v < m.n_p2; ++v)
    if (!m.p2_bnd[v]) map[v] = static_cast<int32_t>(nI++);
  return map;
}

int chunk_size(int remaining) {
  if (remaining >= 8) return 8;
  if (remaining >= 4) return 4;
  if (remaining >= 2) return 2;
  return 1;
}

// Order library work after the caller's stream, and the caller's stream
// after the library work.
struct StreamScope {
  stokes_ctx* c;
  explicit StreamScope(stokes_ctx* cc) : c(cc) {
    HIP_CHECK(hipEventRecord(c->ev_in, c->user_stream));
    HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  }
  ~StreamScope() {
    if (hipEventRecord(c->ev_out, c->stream) == hipSuccess) (void)hipStreamWaitEvent(c->user_stream, c->ev_out, 0);
  }
};

// Zero the outputs of *info; the caller's residual-history buffer and its
// capacity are kept.
void info_reset(stokes_solve_info* info) {
  if (!info) return;
  double* hist = info->res_hist;
  const int32_t cap = info->res_hist_cap;
  std::memset(info, 0, sizeof(*info));
  info->res_hist = hist;
  info->res_hist_cap = hist ? std::max<int32_t>(0, cap) : 0;
}

// Add one batch's counters and residual history to *info.
void info_add(stokes_solve_info* info, const SolveStats& st) {
  if (!info) return;
  info->outer_iters += st.outer;
  info->inner_iters_u += st.inner_u;
  info->inner_iters_p += st.inner_p;
  info->refinements += st.sweeps;
  for (double v : st.hist) {
    if (info->res_hist_len >= info->res_hist_cap) break;
    info->res_hist[info->res_hist_len++] = v;
  }
}

double wall() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void prof_start(stokes_ctx* c, const stokes_solve_opts* o) {
  c->abytes = 0;
  c->prof_on = o->profile;
  c->prof_idx = 0;
  c->prof_seen = 0;
  for (auto& t : c->phase) {
    t.idx = 0;
    t.acc = 0;
  }
  if (c->prof_on && c->prof_ev.empty()) {
    c->prof_ev.resize(16384);
    for (auto& pr : c->prof_ev) {
      HIP_CHECK(hipEventCreate(&pr.first));
      HIP_CHECK(hipEventCreate(&pr.second));
    }
  }
}

void prof_finish(stokes_ctx* c, stokes_solve_info* info) {
  if (info) info->bytes_alg = c->abytes;
  if (!c->prof_on) return;
  HIP_CHECK(hipStreamSynchronize(c->stream));
  double s = 0;
  for (int i = 0; i < c->prof_idx; ++i) {
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, c->prof_ev[i].first, c->prof_ev[i].second));
    s += ms * 1e-3;
  }
  if (info) {
    info->spmv_seconds += s;
    info->spmv_launches += c->prof_idx;
    info->spmv_bytes = c->prof_bytes;
    info->seconds_inner_u = ops::phase_collect(c, PHASE_VEL);
    info->seconds_inner_p = ops::phase_collect(c, PHASE_PRES);
    info->seconds_orth = ops::phase_collect(c, PHASE_ORTH);
  }
  c->prof_on = 0;
}

// Forward solve over batches of right-hand sides.
stokes_status solve_forward(stokes_ctx* c, int method, int32_t nrhs, const double* f, const double* ubc,
                            const double* x0_u, const double* x0_p, double* u, double* p,
                            const stokes_solve_opts* o, stokes_solve_info* info) {
  if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
  if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
  if (!f || !u || !p) throw Error(STOKES_ERR_ARG, "f, u and p must not be NULL");
  if ((x0_u == nullptr) != (x0_p == nullptr)) throw Error(STOKES_ERR_ARG, "x0_u and x0_p must both be given or both NULL");
  check_opts(o);
  info_reset(info);
  const double t0 = wall();
  HIP_CHECK(hipSetDevice(c->device));
  StreamScope scope(c);
  prof_start(c, o);
  const int D = c->dim;
  stokes_status status = STOKES_OK;
  double maxres = 0;
  for (int r0 = 0; r0 < nrhs;) {
    const int nrb = chunk_size(nrhs - r0);
    const int64_t nu = c->n_int * D * nrb, np = c->n_p1 * nrb;
    double* F = static_cast<double*>(c->workspace("abi_F", nu * sizeof(double)));
    double* g = static_cast<double*>(c->workspace("abi_g", np * sizeof(double)));
    // (xu, xp) contiguous: the Krylov updates write the coupled vector in place
    double* xu = static_cast<double*>(c->workspace("abi_x", (nu + np) * sizeof(double)));
    double* xp = xu + nu;
    const int64_t vo = int64_t(r0) * D * c->n_p2, po = int64_t(r0) * c->n_p1;
    ops::rhs(c, nrb, f + vo, ubc ? ubc + vo : nullptr, F, g);
    ops::remove_mean<double>(c, nrb, g);
    if (x0_u) {
      ops::vel_in<double>(c, nrb, x0_u + vo, xu);
      ops::p_in<double>(c, nrb, x0_p + po, xp);
    } else {
      ops::zero_dev(c, xu, nu * sizeof(double));
      ops::zero_dev(c, xp, np * sizeof(double));
    }
    SolveStats st;
    const int s = solve_internal(c, *o, method, nrb, F, g, xu, xp, st, x0_u == nullptr);
    ops::vel_out<double>(c, nrb, xu, ubc ? ubc + vo : nullptr, u + vo, 1);
    ops::p_out<double>(c, nrb, xp, p + po);
    if (s != STOKES_OK) status = s;
    for (double rr : st.rel_res) maxres = std::max(maxres, rr);
    info_add(info, st);
    r0 += nrb;
  }
  HIP_CHECK(hipStreamSynchronize(c->stream));
  prof_finish(c, info);
  if (info) {
    info->converged = status == STOKES_OK ? 1 : 0;
    info->rel_res = maxres;
    info->seconds_total = wall() - t0;
  }
  return status;
}

stokes_status projection_forward(stokes_ctx* c, int32_t nrhs, const double* f, const double* ubc,
                                 const double* p_old, double* u, double* p, const stokes_solve_opts* o,
                                 stokes_solve_info* info) {
  if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
  if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
  if (!f || !u || !p) throw Error(STOKES_ERR_ARG, "f, u and p must not be NULL");
  check_opts(o);
  info_reset(info);
  const double t0 = wall();
  HIP_CHECK(hipSetDevice(c->device));
  StreamScope scope(c);
  prof_start(c, o);
  const int D = c->dim;
  stokes_status status = STOKES_OK;
  double maxres = 0;
  for (int r0 = 0; r0 < nrhs;) {
    const int nrb = chunk_size(nrhs - r0);
    const int64_t nu = c->n_int * D * nrb, np = c->n_p1 * nrb;
    double* F = static_cast<double*>(c->workspace("abi_F", nu * sizeof(double)));
    double* g = static_cast<double*>(c->workspace("abi_g", np * sizeof(double)));
    // (xu, xp) contiguous: the Krylov updates write the coupled vector in place
    double* xu = static_cast<double*>(c->workspace("abi_x", (nu + np) * sizeof(double)));
    double* xp = xu + nu;
    double* po_int = nullptr;
    const int64_t vo = int64_t(r0) * D * c->n_p2, po = int64_t(r0) * c->n_p1;
    ops::rhs(c, nrb, f + vo, ubc ? ubc + vo : nullptr, F, g);
    ops::remove_mean<double>(c, nrb, g);
    if (p_old) {
      po_int = static_cast<double*>(c->workspace("abi_pold", np * sizeof(double)));
      ops::p_in<double>(c, nrb, p_old + po, po_int);
    }
    SolveStats st;
    const int s = projection_internal(c, *o, nrb, F, g, po_int, xu, xp, st);
    ops::vel_out<double>(c, nrb, xu, ubc ? ubc + vo : nullptr, u + vo, 1);
    ops::p_out<double>(c, nrb, xp, p + po);
    if (s != STOKES_OK) status = s;
    for (double rr : st.rel_res) maxres = std::max(maxres, rr);
    info_add(info, st);
    r0 += nrb;
  }
  HIP_CHECK(hipStreamSynchronize(c->stream));
  prof_finish(c, info);
  if (info) {
    info->converged = status == STOKES_OK ? 1 : 0;
    info->rel_res = maxres;
    info->seconds_total = wall() - t0;
  }
  return status;
}

}  // namespace
}  // namespace stokes

using namespace stokes;

void stokes_ctx::clear_graphs() {
  for (auto& kv : graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  graphs.clear();
}

void stokes_ctx::run_graph(const std::string& key, const std::function<void()>& enqueue) {
  if (!use_graphs) {
    enqueue();
    return;
  }
  Graph& g = graphs[key];
  if (g.exec && g.gen == ws_gen) {
    HIP_CHECK(hipGraphLaunch(g.exec, stream));
    abytes += g.bytes;  // the launchers counted the sequence once, at capture
    return;
  }
  if (g.exec) {
    (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
  }
  if (g.eager_runs == 0 || g.gen != ws_gen) {
    // first use (or moved buffers): run eagerly so every workspace exists
    g.gen = ws_gen;
    enqueue();
    g.eager_runs = 1;
    g.gen = ws_gen;
    return;
  }
  const uint64_t gen0 = ws_gen;
  hipGraph_t graph = nullptr;
  const double b0 = abytes;
  HIP_CHECK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue();
  } catch (...) {
    (void)hipStreamEndCapture(stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(stream, &graph));
  g.bytes = abytes - b0;  // counted at capture, moved by the launch below
  if (ws_gen != gen0) throw Error(STOKES_ERR_STATE, "workspace reallocated during graph capture");
  hipGraphExec_t exec = nullptr;
  HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  (void)hipGraphDestroy(graph);
  g.exec = exec;
  g.gen = ws_gen;
  HIP_CHECK(hipGraphLaunch(g.exec, stream));
}

stokes_ctx::~stokes_ctx() {
  clear_graphs();
  if (ev_in) (void)hipEventDestroy(ev_in);
  if (ev_out) (void)hipEventDestroy(ev_out);
  for (auto& pr : prof_ev) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto& t : phase)
    for (auto& pr : t.ev) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (auto& kv : ws_host)
    if (kv.second.first) (void)hipHostFree(kv.second.first);
  if (h_scal) (void)hipHostFree(h_scal);
  ws.clear();
  if (stream) (void)hipStreamDestroy(stream);
}

void* stokes_ctx::workspace_host(const std::string& name, size_t bytes) {
  auto& e = ws_host[name];
  if (e.first && e.second >= bytes) return e.first;
  if (e.first) (void)hipHostFree(e.first);
  e.first = nullptr;
  if (hipHostMalloc(&e.first, bytes, hipHostMallocDefault) != hipSuccess)
    throw Error(STOKES_ERR_ALLOC, "hipHostMalloc failed");
  e.second = bytes;
  return e.first;
}

extern "C" {

void stokes_default_opts(stokes_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = STOKES_FP64;
  o->rtol = 1e-8;
  o->max_outer = 500;
  o->restart = 30;
  o->max_inner = 500;
  o->inner_mode = STOKES_INNER_TOL;
  o->cheb_degree = 4;
  o->inner_rtol_u = 1e-6;
  o->inner_rtol_p = 1e-4;
  o->schur_pc = STOKES_CC_LUMPED;
  o->coupled_pc = STOKES_PC_FULL;
  o->max_refine = 8;
  o->profile = 0;
  o->arnoldi_fp64 = STOKES_ARNOLDI_FP64;
}

const char* stokes_last_error(void) { return g_last_error.c_str(); }

stokes_status stokes_problem_sizes(const stokes_problem* prob, int64_t sizes[10]) {
  return guard([&]() -> stokes_status {
    check_problem(prob);
    if (!sizes) throw Error(STOKES_ERR_ARG, "sizes is NULL");
    HostMesh m;
    if (!build_mesh(prob->dim, prob->n, prob->mesh_seed, prob->jitter, m, order_of(prob)))
      throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large");
    HostCsr P2, B, P1, A2, B2;
    patterns(m, P2, B, P1);
    int64_t nI = 0;
    std::vector<int32_t> imap = interior_map(m, nI);
    std::vector<int32_t> rows_all(m.n_q);
    for (int64_t i = 0; i < m.n_q; ++i) rows_all[i] = static_cast<int32_t>(i);
    restrict_pattern(P2, imap, nI, imap, nI, A2, nullptr);
    restrict_pattern(B, rows_all, m.n_q, imap, nI, B2, nullptr);
    sizes[0] = m.n_p2;
    sizes[1] = m.n_q;
    sizes[2] = nI;
    sizes[3] = A2.rowptr.back();
    sizes[4] = B2.rowptr.back();
    sizes[5] = P1.rowptr.back();
    sizes[6] = m.n_e;
    sizes[7] = m.dim;
    sizes[8] = P2.rowptr.back();
    sizes[9] = B.rowptr.back();
    return STOKES_OK;
  });
}

stokes_status stokes_build_mesh_host(const stokes_problem* prob, double* vcoords, int32_t* elems, double* p2coords,
                                     int32_t* p2) {
  return guard([&]() -> stokes_status {
    check_problem(prob);
    HostMesh m;
    if (!build_mesh(prob->dim, prob->n, prob->mesh_seed, prob->jitter, m, order_of(prob)))
      throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large");
    if (vcoords) std::memcpy(vcoords, m.vcoords.data(), m.vcoords.size() * sizeof(double));
    if (elems) std::memcpy(elems, m.elems.data(), m.elems.size() * sizeof(int32_t));
    if (p2coords) std::memcpy(p2coords, m.p2coords.data(), m.p2coords.size() * sizeof(double));
    if (p2) std::memcpy(p2, m.p2.data(), m.p2.size() * sizeof(int32_t));
    return STOKES_OK;
  });
}

stokes_status stokes_host_pattern(const stokes_problem* prob, int32_t which, int64_t* nrows, int64_t* nnz,
                                  int32_t* rowptr, int32_t* cols) {
  return guard([&]() -> stokes_status {
    check_problem(prob);
    if (which < 0 || which > 4) throw Error(STOKES_ERR_ARG, "which must be in [0, 4]");
    if (!nrows || !nnz) throw Error(STOKES_ERR_ARG, "nrows and nnz must not be NULL");
    HostMesh m;
    if (!build_mesh(prob->dim, prob->n, prob->mesh_seed, prob->jitter, m, order_of(prob)))
      throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large");
    HostCsr P2, B, P1, out;
    patterns(m, P2, B, P1);
    int64_t nI = 0;
    std::vector<int32_t> imap = interior_map(m, nI);
    std::vector<int32_t> rows_all(m.n_q);
    for (int64_t i = 0; i < m.n_q; ++i) rows_all[i] = static_cast<int32_t>(i);
    const HostCsr* h = nullptr;
    switch (which) {
      case 0: h = &P2; break;
      case 1: restrict_pattern(P2, imap, nI, imap, nI, out, nullptr); h = &out; break;
      case 2: h = &B; break;
      case 3: restrict_pattern(B, rows_all, m.n_q, imap, nI, out, nullptr); h = &out; break;
      default: h = &P1; break;
    }
    *nrows = h->nrows;
    *nnz = h->rowptr.back();
    if (rowptr && cols) {
      for (int64_t i = 0; i <= h->nrows; ++i) rowptr[i] = static_cast<int32_t>(h->rowptr[i]);
      std::memcpy(cols, h->cols.data(), h->cols.size() * sizeof(int32_t));
    }
    return STOKES_OK;
  });
}

stokes_status stokes_assemble(const stokes_problem* prob, void* hip_stream, stokes_ctx** out) {
  return guard([&]() -> stokes_status {
    check_problem(prob);
    if (!out) throw Error(STOKES_ERR_ARG, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      throw Error(STOKES_ERR_HIP, "no HIP device available");
    }
    auto c = std::make_unique<stokes_ctx>();
    c->prob = *prob;
    c->strain = (prob->flags & STOKES_FLAG_STRAIN) != 0;
    HIP_CHECK(hipGetDevice(&c->device));
    (void)scratch_on(c->device);  // set-up of the allocation-free residual, once per device
    c->user_stream = static_cast<hipStream_t>(hip_stream);
    if (const char* e = std::getenv("STOKES_GRAPHS")) c->use_graphs = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_CG_CHECK")) c->cg_check_every = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("STOKES_MGX")) c->use_mgx = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_MGX_P3")) c->mgx_p3 = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_MGX_P2_RATIO")) c->mgx_p2_ratio = std::max(1.5, std::atof(e));
    if (const char* e = std::getenv("STOKES_MGX_P2_DEGREE")) c->mgx_p2_degree = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("STOKES_VEL_HALF")) c->vel_half = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_PMG_HALF")) c->pmg_half = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_VEL_BF")) c->vel_bf = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_VEL_IL")) c->vel_il = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_VEL_AF")) c->vel_af = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_CHEB_DEFER")) c->cheb_defer = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_GRAM")) c->gram_cgs2 = std::atoi(e) != 0;
    if (const char* e = std::getenv("STOKES_LANES")) c->force_lanes = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("STOKES_ZBLOCK")) c->zblock = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("STOKES_VEL_PAIR")) c->vel_pair = std::max(0, std::min(2, std::atoi(e)));
    if (const char* e = std::getenv("STOKES_SLICE_YQ")) c->slice_yq = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("STOKES_SLICE_SCHED")) c->slice_sched = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("STOKES_MG_ES")) {
      const int v = std::atoi(e);
      c->mg_es = (v == -1 || v == 0 || v == 2 || v == 4 || v == 8 || v == 16) ? v : 1;
    }
    if (const char* e = std::getenv("STOKES_MG_DEGREE")) c->mg_smooth_degree = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("STOKES_MG_RATIO")) c->mg_smooth_ratio = std::max(1.5, std::atof(e));
    HIP_CHECK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIP_CHECK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIP_CHECK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    HIP_CHECK(hipStreamSynchronize(c->user_stream));
    if (!build_mesh(prob->dim, prob->n, prob->mesh_seed, prob->jitter, c->mesh, order_of(prob)))
      throw Error(STOKES_ERR_UNSUPPORTED, "mesh too large");
    c->dim = prob->dim;
    c->nloc = c->mesh.nloc;
    c->n_p1 = c->mesh.n_q;  // pressure nodes
    c->n_p2 = c->mesh.n_p2;
    c->n_e = c->mesh.n_e;
    c->red.partials.alloc(size_t(kMaxBlocks) * 2 * kMaxSys * sizeof(double));
    c->red.ticket.alloc(64);
    HIP_CHECK(hipMemset(c->red.ticket.p, 0, 64));
    c->red.result.alloc(8 * kMaxSys * sizeof(double));
    c->scal.alloc(4 * sizeof(Scalars));
    HIP_CHECK(hipMemset(c->scal.p, 0, 4 * sizeof(Scalars)));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_scal), sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
      throw Error(STOKES_ERR_ALLOC, "hipHostMalloc failed");
    c->ones64.alloc(c->n_p1 * 8 * sizeof(double));
    c->ones32.alloc(c->n_p1 * 8 * sizeof(float));
    hipLaunchKernelGGL(k_set<double>, dim3(ops::grid_for(c->n_p1 * 8)), dim3(kBlock), 0, c->stream, c->n_p1 * 8, 1.0,
                       c->ones64.as<double>());
    hipLaunchKernelGGL(k_set<float>, dim3(ops::grid_for(c->n_p1 * 8)), dim3(kBlock), 0, c->stream, c->n_p1 * 8, 1.0f,
                       c->ones32.as<float>());
    ops::check_launch();
    assemble_ctx(c.get());
    *out = c.release();
    return STOKES_OK;
  });
}

stokes_status stokes_solve_schur(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                                 const double* x0_u, const double* x0_p, double* u, double* p,
                                 const stokes_solve_opts* opts, stokes_solve_info* info) {
  return guard([&]() { return solve_forward(ctx, 1, nrhs, f, ubc, x0_u, x0_p, u, p, opts, info); });
}

stokes_status stokes_solve_coupled(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                                   const double* x0_u, const double* x0_p, double* u, double* p,
                                   const stokes_solve_opts* opts, stokes_solve_info* info) {
  return guard([&]() { return solve_forward(ctx, 0, nrhs, f, ubc, x0_u, x0_p, u, p, opts, info); });
}

stokes_status stokes_projection_step(stokes_ctx* ctx, int32_t nrhs, const double* f, const double* ubc,
                                     const double* p_old, double* u, double* p, const stokes_solve_opts* opts,
                                     stokes_solve_info* info) {
  return guard([&]() { return projection_forward(ctx, nrhs, f, ubc, p_old, u, p, opts, info); });
}

stokes_status stokes_solve_adjoint(stokes_ctx* c, int32_t nrhs, const double* u, const double* dJdu,
                                   const double* dJdp, double* lam_u, double* lam_p, double* dJdf, double* dJdmu,
                                   const stokes_solve_opts* o, stokes_solve_info* info) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
    if (!u || !dJdu || !lam_u || !lam_p || !dJdf || !dJdmu) throw Error(STOKES_ERR_ARG, "NULL array argument");
    check_opts(o);
    info_reset(info);
    const double t0 = wall();
    HIP_CHECK(hipSetDevice(c->device));
    StreamScope scope(c);
    prof_start(c, o);
    const int D = c->dim;
    stokes_status status = STOKES_OK;
    double maxres = 0;
    for (int r0 = 0; r0 < nrhs;) {
      const int nrb = chunk_size(nrhs - r0);
      const int64_t nu = c->n_int * D * nrb, np = c->n_p1 * nrb;
      double* F = static_cast<double*>(c->workspace("abi_F", nu * sizeof(double)));
      double* g = static_cast<double*>(c->workspace("abi_g", np * sizeof(double)));
      double* xu = static_cast<double*>(c->workspace("abi_x", (nu + np) * sizeof(double)));
      double* xp = xu + nu;
      const int64_t vo = int64_t(r0) * D * c->n_p2, po = int64_t(r0) * c->n_p1;
      // j_u = dJ/dU on the interior; the pressure part is Pi^T dJdp with Pi the
      // zero-integral normalisation, then negated (lam_p -> -lam_p turns the
      // transposed system into the forward one)
      ops::vel_in<double>(c, nrb, dJdu + vo, F);
      if (dJdp) {
        ops::p_in<double>(c, nrb, dJdp + po, g);
        ops::adj_jp(c, nrb, g);
      } else {
        ops::zero_dev(c, g, np * sizeof(double));
      }
      ops::zero_dev(c, xu, nu * sizeof(double));
      ops::zero_dev(c, xp, np * sizeof(double));
      SolveStats st;
      const int s = solve_internal(c, *o, 0, nrb, F, g, xu, xp, st, true);
      if (s != STOKES_OK) status = s;
      for (double rr : st.rel_res) maxres = std::max(maxres, rr);
      // lam_p = -q
      ops::axpby<double>(c, np, 0.0, xp, -1.0, xp);
      ops::vel_out<double>(c, nrb, xu, nullptr, lam_u + vo, 1);
      ops::p_out<double>(c, nrb, xp, lam_p + po);
      ops::adj_dJdf(c, nrb, xu, dJdf + vo);
      ops::adj_dJdmu(c, nrb, u + vo, xu, c->red.result.as<double>() + 4 * kMaxSys);
      HIP_CHECK(hipMemcpyAsync(dJdmu + r0, c->red.result.as<double>() + 4 * kMaxSys, nrb * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
      info_add(info, st);
      r0 += nrb;
    }
    HIP_CHECK(hipStreamSynchronize(c->stream));
    prof_finish(c, info);
    if (info) {
      info->converged = status == STOKES_OK ? 1 : 0;
      info->rel_res = maxres;
      info->seconds_total = wall() - t0;
    }
    return status;
  });
}

stokes_status stokes_apply(stokes_ctx* c, int32_t op, int32_t precision, int32_t nrhs, const double* x, double* y) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (op < 0 || op > 10) throw Error(STOKES_ERR_ARG, "op must be in [0, 10]");
    if (precision != 0 && precision != 1) throw Error(STOKES_ERR_ARG, "precision must be 0 or 1");
    if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
    if (!x || !y) throw Error(STOKES_ERR_ARG, "x and y must not be NULL");
    if (c->mesh.order == 3 && op == 9)
      throw Error(STOKES_ERR_UNSUPPORTED, "the velocity multigrid (op 9) needs the P2/P1 pair");
    if (op == 8 && c->mgx.lv.empty())
      throw Error(STOKES_ERR_UNSUPPORTED, "no Galerkin pressure multigrid on this context (STOKES_MGX_P3=0)");
    HIP_CHECK(hipSetDevice(c->device));
    StreamScope scope(c);
    const int D = c->dim;
    for (int r0 = 0; r0 < nrhs;) {
      const int nrb = chunk_size(nrhs - r0);
      const int64_t nu = c->n_int * D * nrb, np = c->n_p1 * nrb;
      const int64_t vo = int64_t(r0) * D * c->n_p2, po = int64_t(r0) * c->n_p1;
      const int64_t tot_u = int64_t(nrhs) * D * c->n_p2;
      double* xu = static_cast<double*>(c->workspace("ap_xu", nu * sizeof(double)));
      double* xp = static_cast<double*>(c->workspace("ap_xp", np * sizeof(double)));
      double* yu = static_cast<double*>(c->workspace("ap_yu", nu * sizeof(double)));
      double* yp = static_cast<double*>(c->workspace("ap_yp", np * sizeof(double)));
      float* xuf = static_cast<float*>(c->workspace("ap_xuf", nu * sizeof(float)));
      float* xpf = static_cast<float*>(c->workspace("ap_xpf", np * sizeof(float)));
      float* yuf = static_cast<float*>(c->workspace("ap_yuf", nu * sizeof(float)));
      float* ypf = static_cast<float*>(c->workspace("ap_ypf", np * sizeof(float)));
      const bool in_vel = op == 0 || op == 1 || op == 5 || op == 9 || op == 10;
      const bool in_p = op == 2 || op == 3 || op == 4 || op == 5 || op == 6 || op == 7 || op == 8;
      const bool out_vel = op == 0 || op == 2 || op == 5 || op == 9 || op == 10;
      const double* xv = x + vo;
      const double* xpp = op == 5 ? x + tot_u + po : x + po;
      if (in_vel) ops::vel_in<double>(c, nrb, xv, xu);
      if (in_p) ops::p_in<double>(c, nrb, xpp, xp);
      if (precision == 1) {
        if (in_vel) ops::cast<double, float>(c, nu, xu, xuf);
        if (in_p) ops::cast<double, float>(c, np, xp, xpf);
      }
      auto run = [&](auto tag, auto* XU, auto* XP, auto* YU, auto* YP) {
        using T = std::remove_pointer_t<decltype(XU)>;
        (void)tag;
        switch (op) {
          case 0: ops::velop<T>(c, nrb, XU, YU, (T)1, nullptr, (T)0); break;
          case 1: ops::Bmul<T>(c, nrb, XU, YP, (T)1, nullptr, (T)0); break;
          case 2: ops::Btmul<T>(c, nrb, XP, nullptr, YU, (T)1, nullptr, (T)0); break;
          case 3: ops::spmv<T>(c, c->sQ, ops::pick<T>(c->MQ64, c->MQ32), nrb, XP, YP, (T)1, nullptr, (T)0); break;
          case 4: ops::spmv<T>(c, c->sQ, ops::pick<T>(c->LQ64, c->LQ32), nrb, XP, YP, (T)1, nullptr, (T)0); break;
          case 6: mg_vcycle<T>(c, c->mgq, nrb, XP, YP, 0); break;
          case 8: mg_vcycle<T>(c, c->mgx, nrb, XP, YP, 0); break;
          case 9: vel_vcycle<T>(c, D * nrb, XU, YU, 0); break;
          case 10: vel_cheb_apply<T>(c, nrb, 6, XU, YU); break;
          case 7: ops::spmv<T>(c, c->sX, ops::pick<T>(c->XL64, c->XL32), nrb, XP, YP, (T)1, nullptr, (T)0); break;
          default:
            ops::momentum<T>(c, nrb, XU, XP, nullptr, YU, (T)1, nullptr);
            ops::Bmul<T>(c, nrb, XU, YP, (T)1, nullptr, (T)0);
        }
      };
      ops::ensure_lanes(c, D * nrb, precision == 1);
      if (op == 9 && (!c->vmg_built || c->vmg_mu != c->prob.mu)) build_vmg(c);
      if (precision == 1) run(0, xuf, xpf, yuf, ypf);
      else run(0, xu, xp, yu, yp);
      if (precision == 1) {
        if (out_vel) ops::cast<float, double>(c, nu, yuf, yu);
        if (!out_vel || op == 5) ops::cast<float, double>(c, np, ypf, yp);
      }
      if (out_vel) ops::vel_out<double>(c, nrb, yu, nullptr, y + vo, 1);
      if (!out_vel || op == 5) ops::p_out<double>(c, nrb, yp, op == 5 ? y + tot_u + po : y + po);
      r0 += nrb;
    }
    HIP_CHECK(hipStreamSynchronize(c->stream));
    return STOKES_OK;
  });
}

stokes_status stokes_residual(stokes_ctx* c, int32_t nrhs, const double* f, const double* ubc, const double* u,
                              const double* p, double* rel) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
    if (!f || !u || !p || !rel) throw Error(STOKES_ERR_ARG, "NULL array argument");
    HIP_CHECK(hipSetDevice(c->device));
    StreamScope scope(c);
    const int D = c->dim;
    for (int r0 = 0; r0 < nrhs;) {
      const int nrb = chunk_size(nrhs - r0);
      const int64_t nu = c->n_int * D * nrb, np = c->n_p1 * nrb;
      const int64_t vo = int64_t(r0) * D * c->n_p2, po = int64_t(r0) * c->n_p1;
      double* F = static_cast<double*>(c->workspace("rs_F", nu * sizeof(double)));
      double* g = static_cast<double*>(c->workspace("rs_g", np * sizeof(double)));
      double* xu = static_cast<double*>(c->workspace("rs_xu", nu * sizeof(double)));
      double* xp = static_cast<double*>(c->workspace("rs_xp", np * sizeof(double)));
      double* ru = static_cast<double*>(c->workspace("rs_ru", nu * sizeof(double)));
      double* rp = static_cast<double*>(c->workspace("rs_rp", np * sizeof(double)));
      ops::rhs(c, nrb, f + vo, ubc ? ubc + vo : nullptr, F, g);
      ops::remove_mean<double>(c, nrb, g);
      ops::vel_in<double>(c, nrb, u + vo, xu);
      ops::p_in<double>(c, nrb, p + po, xp);
      ops::momentum<double>(c, nrb, xu, xp, nullptr, ru, -1.0, F);
      ops::Bmul<double>(c, nrb, xu, rp, -1.0, g, 1.0);
      auto s1 = ops::dot_host<double>(c, c->n_int, D * nrb, ru, ru);
      auto s2 = ops::dot_host<double>(c, c->n_p1, nrb, rp, rp);
      auto b1 = ops::dot_host<double>(c, c->n_int, D * nrb, F, F);
      auto b2 = ops::dot_host<double>(c, c->n_p1, nrb, g, g);
      for (int r = 0; r < nrb; ++r) {
        double num = s2[r], den = b2[r];
        for (int d = 0; d < D; ++d) {
          num += s1[r * D + d];
          den += b1[r * D + d];
        }
        rel[r0 + r] = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
      }
      r0 += nrb;
    }
    return STOKES_OK;
  });
}

stokes_status stokes_residual_noalloc(stokes_ctx* c, int32_t nrhs, const double* f, const double* ubc,
                                      const double* u, const double* p, double* rel) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (nrhs < 1) throw Error(STOKES_ERR_ARG, "nrhs must be >= 1");
    if (!f || !u || !p || !rel) throw Error(STOKES_ERR_ARG, "NULL array argument");
    const int D = c->dim;
    const int64_t nu = c->n_int * D, np = c->n_p1;  // one right-hand side at a time
    const size_t need = size_t(2 * nu + 2 * np) * sizeof(double);
    if (need > kScratchBytes)
      throw Error(STOKES_ERR_UNSUPPORTED, "stokes_residual_noalloc needs " + std::to_string(need) +
                                              " bytes of scratch for this mesh; the limit is " +
                                              std::to_string(kScratchBytes) + " (use stokes_residual)");
    HIP_CHECK(hipSetDevice(c->device));
    double* base = static_cast<double*>(scratch_on(c->device));
    StreamScope scope(c);
    // [F | xu | g | xp]: the residual overwrites (F, g) in place; xu first
    // stages the interior forcing.  Every slot is fully written before it is
    // read, so nothing left by an earlier call is used.
    double* F = base;
    double* xu = F + nu;
    double* g = xu + nu;
    double* xp = g + np;
    double* res = c->red.result.as<double>();
    double h[2 * 3 + 2];
    for (int r = 0; r < nrhs; ++r) {
      const int64_t vo = int64_t(r) * D * c->n_p2, po = int64_t(r) * c->n_p1;
      ops::rhs(c, 1, f + vo, ubc ? ubc + vo : nullptr, F, g, xu);
      ops::remove_mean<double>(c, 1, g);
      ops::vel_in<double>(c, 1, u + vo, xu);
      ops::p_in<double>(c, 1, p + po, xp);
      ops::dot_dev<double>(c, c->n_int, D, F, F, nullptr, res);
      ops::dot_dev<double>(c, c->n_p1, 1, g, g, nullptr, res + D);
      ops::momentum<double>(c, 1, xu, xp, nullptr, F, -1.0, F);  // r_u = F - (A u - B^T p)
      ops::Bmul<double>(c, 1, xu, g, -1.0, g, 1.0);              // r_p = g - B u
      ops::dot_dev<double>(c, c->n_int, D, F, F, nullptr, res + D + 1);
      ops::dot_dev<double>(c, c->n_p1, 1, g, g, nullptr, res + 2 * D + 1);
      HIP_CHECK(hipMemcpyAsync(h, res, (2 * D + 2) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
      HIP_CHECK(hipStreamSynchronize(c->stream));
      double den = h[D], num = h[2 * D + 1];
      for (int d = 0; d < D; ++d) {
        den += h[d];
        num += h[D + 1 + d];
      }
      rel[r] = den > 0 ? std::sqrt(num / den) : std::sqrt(num);
    }
    return STOKES_OK;
  });
}

}  // extern "C"

namespace stokes {
namespace {

// Bandwidth probe kernels: 16-byte nontemporal streams, grid-stride.
typedef unsigned probe_u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_probe_copy(int64_t n16, const probe_u32x4* __restrict__ src,
                                                       probe_u32x4* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Read stream: every word is summed (xor) so the loads stay; one word per
// block is written.
__global__ __launch_bounds__(kBlock) void k_probe_read(int64_t n16, const probe_u32x4* __restrict__ src,
                                                       unsigned* __restrict__ out) {
  unsigned acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n16; i += (int64_t)gridDim.x * kBlock) {
    const probe_u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)] = acc;
}

}  // namespace
}  // namespace stokes

extern "C" {

stokes_status stokes_bandwidth_probe(void* hip_stream, int64_t bytes, int32_t reps, double* gbs_host) {
  return guard([&]() -> stokes_status {
    if (bytes < (int64_t(1) << 20) || bytes > (int64_t(1) << 36) || reps < 1 || reps > 100 || !gbs_host)
      throw Error(STOKES_ERR_ARG, "bytes must be in [1 MiB, 64 GiB], reps in [1, 100], gbs_host non-NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t n16 = bytes / 16;
    DevBuf a, b, o;
    a.alloc(n16 * 16);
    b.alloc(n16 * 16);
    const int nblk = 8 * 256 * 4;  // 4 workgroups of 256 threads per CU on 256 CUs, x2
    o.alloc(size_t(nblk) * (kBlock / 64) * sizeof(unsigned));
    HIP_CHECK(hipMemsetAsync(a.p, 1, n16 * 16, s));
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    struct Ev {
      hipEvent_t a, b;
      ~Ev() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } guard_ev{e0, e1};
    auto timed = [&](auto launch) {
      launch();  // warm-up
      HIP_CHECK(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) launch();
      HIP_CHECK(hipEventRecord(e1, s));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      return ms * 1e-3 / reps;
    };
    const double tc = timed([&] {
      hipLaunchKernelGGL(k_probe_copy, dim3(nblk), dim3(kBlock), 0, s, n16, a.as<const probe_u32x4>(), b.as<probe_u32x4>());
    });
    const double tr = timed([&] {
      hipLaunchKernelGGL(k_probe_read, dim3(nblk), dim3(kBlock), 0, s, n16, a.as<const probe_u32x4>(), o.as<unsigned>());
    });
    HIP_CHECK(hipGetLastError());
    gbs_host[0] = 2.0 * double(n16 * 16) / tc * 1e-9;
    gbs_host[1] = double(n16 * 16) / tr * 1e-9;
    HIP_CHECK(hipStreamSynchronize(s));
    return STOKES_OK;
  });
}

stokes_status stokes_query(const stokes_ctx* c, int64_t sizes[12]) {
  return guard([&]() -> stokes_status {
    if (!c || !sizes) throw Error(STOKES_ERR_ARG, "NULL argument");
    sizes[0] = c->n_p2;
    sizes[1] = c->n_p1;
    sizes[2] = c->n_int;
    sizes[3] = c->sA.nnz;
    sizes[4] = c->sB.nnz;
    sizes[5] = c->sQ.nnz;
    sizes[6] = c->n_e;
    sizes[7] = c->dim;
    sizes[8] = c->p2full.nnz;
    sizes[9] = c->bfull.nnz;
    sizes[10] = c->xl.nnz;
    sizes[11] = c->vel_af ? c->sA.affine_slices : 0;
    return STOKES_OK;
  });
}

stokes_status stokes_set_mu(stokes_ctx* c, double mu) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (!(mu > 0) || !std::isfinite(mu)) throw Error(STOKES_ERR_ARG, "mu must be finite and > 0");
    HIP_CHECK(hipSetDevice(c->device));
    c->prob.mu = mu;
    reform_A(c);
    return STOKES_OK;
  });
}

stokes_status stokes_set_stream(stokes_ctx* c, void* stream) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    HIP_CHECK(hipStreamSynchronize(c->stream));
    c->user_stream = static_cast<hipStream_t>(stream);
    return STOKES_OK;
  });
}

stokes_status stokes_export_mesh(const stokes_ctx* c, double* p2coords, int32_t* p2) {
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (p2coords) std::memcpy(p2coords, c->mesh.p2coords.data(), c->mesh.p2coords.size() * sizeof(double));
    if (p2) std::memcpy(p2, c->mesh.p2.data(), c->mesh.p2.size() * sizeof(int32_t));
    return STOKES_OK;
  });
}

stokes_status stokes_export_csr(const stokes_ctx* cc, int32_t which, int32_t* rowptr, int32_t* cols, double* vals) {
  stokes_ctx* c = const_cast<stokes_ctx*>(cc);
  return guard([&]() -> stokes_status {
    if (!c) throw Error(STOKES_ERR_ARG, "ctx is NULL");
    if (which < 0 || which > 9 + c->dim * c->dim) throw Error(STOKES_ERR_ARG, "which out of range");
    if (which >= 10 && !c->strain) throw Error(STOKES_ERR_STATE, "grad-div blocks exist only with STOKES_FLAG_STRAIN");
    if (!vals) throw Error(STOKES_ERR_ARG, "vals is NULL");
    HIP_CHECK(hipSetDevice(c->device));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    auto copy_csr = [&](const DevCsr& P, const DevBuf& v, int planes, int plane) {
      if (rowptr) HIP_CHECK(hipMemcpy(rowptr, P.rowptr.p, (P.nrows + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
      if (cols) HIP_CHECK(hipMemcpy(cols, P.cols.p, P.nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
      std::vector<double> h(P.nnz * planes);
      HIP_CHECK(hipMemcpy(h.data(), v.p, h.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t k = 0; k < P.nnz; ++k) vals[k] = h[k * planes + plane];
    };
    switch (which) {
      case 0: copy_csr(c->p2full, c->M_full, 1, 0); break;
      case 1: copy_csr(c->p2full, c->L_full, 1, 0); break;
      case 2:
      case 3:
      case 4:
        if (which - 2 >= c->dim) throw Error(STOKES_ERR_ARG, "no such B plane");
        copy_csr(c->bfull, c->B_full, c->dim, which - 2);
        break;
      case 5: copy_csr(c->p1, c->MQ_csr, 1, 0); break;
      case 6: copy_csr(c->p1, c->LQ_csr, 1, 0); break;
      case 9: copy_csr(c->xl, c->XL_csr, 1, 0); break;
      case 10: case 11: case 12: case 13: case 14: case 15: case 16: case 17: case 18:
        copy_csr(c->p2full, c->D_full, c->dim * c->dim, which - 10);
        break;
      case 7: {
        // A_II in the natural interior numbering (pattern 1 of stokes_host_pattern)
        const Sell& S = c->sA;
        std::vector<int64_t> sp(S.nslices + 1);
        std::vector<int32_t> sc(S.nnz_pad);
        std::vector<double> sv(S.nnz_pad);
        HIP_CHECK(hipMemcpy(sp.data(), S.slice_ptr.p, sp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(sc.data(), S.cols.p, sc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        HIP_CHECK(hipMemcpy(sv.data(), c->A64.p, sv.size() * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<int32_t> srcv(S.nnz_pad);
        HIP_CHECK(hipMemcpy(srcv.data(), S.src.p, srcv.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        // natural interior index of every internal row
        std::vector<int32_t> nat_rank(c->n_p2, -1);
        int32_t k = 0;
        for (int64_t v = 0; v < c->n_p2; ++v)
          if (c->h_nat2int[v] >= 0) nat_rank[v] = k++;
        std::vector<std::vector<std::pair<int32_t, double>>> rows(c->n_int);
        for (int64_t r = 0; r < S.nrows; ++r) {
          const int64_t s = r / 64, l = r % 64;
          const int32_t nr = nat_rank[c->h_int2nat[r]];
          for (int64_t q = sp[s] + l; q < sp[s + 1]; q += 64)
            if (srcv[q] >= 0) rows[nr].emplace_back(nat_rank[c->h_int2nat[sc[q]]], sv[q]);
        }
        int64_t o = 0;
        if (rowptr) rowptr[0] = 0;
        for (int64_t r = 0; r < c->n_int; ++r) {
          std::sort(rows[r].begin(), rows[r].end());
          for (auto& e : rows[r]) {
            if (cols) cols[o] = e.first;
            vals[o] = e.second;
            ++o;
          }
          if (rowptr) rowptr[r + 1] = static_cast<int32_t>(o);
        }
        break;
      }
      case 8:
        HIP_CHECK(hipMemcpy(vals, c->lam_full.p, c->n_p2 * sizeof(double), hipMemcpyDeviceToHost));
        break;
      default:
        break;
    }
    return STOKES_OK;
  });
}

stokes_status stokes_bounds(const stokes_ctx* c, double b[8]) {
  return guard([&]() -> stokes_status {
    if (!c || !b) throw Error(STOKES_ERR_ARG, "NULL argument");
    b[0] = c->bA.lo;
    b[1] = c->bA.hi;
    b[2] = c->bMV.lo;
    b[3] = c->bMV.hi;
    b[4] = c->bMQ.lo;
    b[5] = c->bMQ.hi;
    b[6] = c->bXQ.lo;
    b[7] = c->bXQ.hi;
    return STOKES_OK;
  });
}

void stokes_destroy(stokes_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  delete c;
}

}  // extern "C"

// Internal declarations shared by the HIP translation units of libstokes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/stokes.h"
#include "mesh_host.h"

namespace stokes {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  stokes_status code;
  Error(stokes_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_CHECK(expr)                                                                        \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw ::stokes::Error(STOKES_ERR_HIP, std::string(#expr " failed: ") + hipGetErrorString(e_) + \
                                                " (" __FILE__ ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

void set_last_error(const std::string& msg);

// --------------------------------------------------------- device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();
  void alloc(size_t b);          // exact size, contents undefined
  void ensure(size_t b);         // grow-only
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
void upload(DevBuf& b, const std::vector<T>& v) {
  b.alloc(std::max<size_t>(1, v.size()) * sizeof(T));
  if (!v.empty()) HIP_CHECK(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

// Sliced ELL with slice height 64 (one wavefront), one thread per row.
// Entry j of row r (slice s = r / 64, lane l = r % 64) sits at
// slice_ptr[s] + 64 j + l; padding entries have value 0 (src -1) and the
// column of a neighbouring lane's entry in the same slot (0 if none).
// Device view of the column indices of a Sell (see slice_ref in kernels.h).
struct SellIdx {
  const int64_t* sp = nullptr;     // slice_ptr
  const int32_t* cols = nullptr;   // 32-bit columns (slices with pk = 0)
  const int32_t* cbase = nullptr;  // [nnz_pad / 64] base column of slot j of slice s at sp[s] / 64 + j
  const uint8_t* cdel = nullptr;   // [nnz_pad] column - base (slices with pk = 1)
  const int32_t* pk = nullptr;     // [nslices] 1 = packed columns, 2 = packed and affine (32-bit: a scalar load)
  // [2 per slot] affine slots: column of lane l = base + l + (l >= brk ? jump : 0),
  // stored as (base, brk | jump << 8); null: kernels read the packed offsets
  const int32_t* cmeta = nullptr;
  // [nslices] slice schedule of the gathering kernels (XCD_ROWS_G): the t-th
  // slice of an eighth of the rows in launch order is rperm[t], a slice of
  // the same eighth; null: slice order
  const int32_t* rperm = nullptr;
};

constexpr int kSchedMinW = 12;  // narrowest product (values per row) launched in the slice schedule

struct Sell {
  int64_t nrows = 0, nslices = 0, nnz = 0, nnz_pad = 0;
  int64_t packed_slices = 0, affine_slices = 0;
  double idx_bytes = 0;     // bytes of the column-index structure streamed by one product
  double idx_bytes_af = 0;  // ... by a product that computes the affine slots' columns
  int64_t ncols = 0;        // columns (rows of a gathered vector)
  int planes = 1;       // values per entry (B and B^T carry dim planes)
  int es = 1;           // lanes sharing a row in the scalar products (1: one lane per row; tuned per MG level)
  DevBuf slice_ptr;     // int64 [nslices + 1]
  DevBuf cols;          // int32 [nnz_pad]
  DevBuf src;           // int32 [nnz_pad] source entry in the assembled CSR (-1 = pad)
  DevBuf cbase, cdel, pk, cmeta;
  const int32_t* rperm = nullptr;  // slice schedule (not owned; the velocity-row patterns share one)
  // the index as a kernel with W values per row reads it: the slice schedule
  // only for W >= kSchedMinW (narrower products lose more to the lookup
  // before each wavefront's first load than they gain in L2 reuse)
  SellIdx idx(int W = 0) const {
    return SellIdx{slice_ptr.as<const int64_t>(), cols.as<const int32_t>(), cbase.as<const int32_t>(),
                   cdel.as<const uint8_t>(), pk.as<const int32_t>(), cmeta.as<const int32_t>(),
                   W >= kSchedMinW ? rperm : nullptr};
  }
};

struct DevCsr {
  int64_t nrows = 0, nnz = 0;
  DevBuf rowptr;  // int32 [nrows + 1]
  DevBuf cols;    // int32 [nnz]
};

// Chebyshev interval of a Jacobi-scaled SPD operator.
struct Bounds {
  double lo = 0, hi = 0;
};

// Reduction scratch for one-pass grid reductions (per context / stream).
struct RedScratch {
  DevBuf partials;  // double [max_blocks * max_slots]
  DevBuf ticket;    // unsigned
  DevBuf result;    // double [max_slots], last reduction result
};

constexpr int kMaxSys = 24;   // systems per batched solve (dim * rhs)
constexpr int kMaxBlocks = 2048;
constexpr int kBlock = 256;

// One level of a pressure multigrid hierarchy, owned by the hierarchy.
struct MgLevel {
  int n = 0;            // cells per side
  int64_t nrows = 0;    // (n + 1)^dim vertices
  Sell S;               // SELL pattern of the level operator
  DevBuf v64, v32;      // operator values
  DevBuf v16;           // FP32 V-cycles: half-precision values / s16 (empty: none)
  float s16 = 0;
  DevBuf d64, d32;      // inverse diagonal
  Bounds bs, bf;        // smoothing interval, full spectrum
};

// One coarse level of the velocity multigrid (scalar alpha M + mu L on the
// interior P2 nodes of the Kuhn mesh with n cells per side, natural order).
struct VmgLevel {
  int n = 0;
  int64_t nrows = 0;
  Sell S;
  DevBuf v64, v32, d64, d32;  // operator values and inverse diagonal
  Bounds bs, bf;              // smoothing interval, full spectrum
  // interpolation from this level to the next finer one: P (fine rows x
  // nrows) and its transpose R, FP64 and FP32 values
  DevCsr P, R;
  DevBuf pv64, pv32, rv64, rv32;
};

// A multigrid hierarchy on the nested Kuhn meshes n, n/2, ...  Level views
// point either at context-owned operators or at levels in `own`.
struct MgHier {
  struct View {
    const Sell* S;
    const DevBuf *v64, *v32, *d64, *d32;
    const Bounds *bs, *bf;
    int n;
    const DevBuf* v16 = nullptr;  // half-precision values / s16 (FP32 V-cycles)
    float s16 = 0;
    int nu = 0;  // smoothing degree of this level (0: the context's)
  };
  std::vector<View> lv;
  std::vector<std::unique_ptr<MgLevel>> own;
  int64_t dense_n = 0;        // > 0: the coarsest level is solved by a dense inverse
  DevBuf cinv64, cinv32;      // [n][n] inverse of the coarsest operator
};

// GPU time of one solver phase, from pairs of HIP events recorded on the
// solver stream around each application (opts.profile = 2 only).
struct PhaseTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  int idx = 0;       // pairs recorded since the last collection
  double acc = 0;    // seconds collected so far in this call
};
enum { PHASE_VEL = 0, PHASE_PRES = 1, PHASE_ORTH = 2, NUM_PHASES = 3 };

// Per-solver device scalars (one set per Krylov instance).
struct Scalars {
  double rho[kMaxSys], rho_old[kMaxSys], alpha[kMaxSys], beta[kMaxSys];
  double sigma[kMaxSys], rr[kMaxSys], bb[kMaxSys], tol2[kMaxSys];
  int active[kMaxSys];
  int breakdown;
};

}  // namespace stokes

struct stokes_ctx {
  stokes_problem prob{};
  hipStream_t stream = nullptr;       // library-owned stream (all work; capturable)
  hipStream_t user_stream = nullptr;  // caller's stream, ordered with `stream` by events
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int device = 0;
  int dim = 0, nloc = 0;
  int64_t n_p1 = 0, n_p2 = 0, n_e = 0, n_int = 0;

  stokes::HostMesh mesh;  // kept for export

  // full-numbering CSR matrices (assembly products)
  stokes::DevCsr p2full, bfull, p1;
  stokes::DevCsr xl;              // P1 x P1 pattern of B_I Lambda_V^-1 B_I^T
  // interior rows with boundary neighbours: internal row ids, CSR over their
  // boundary columns (natural ids) and the entry index in the p2full pattern
  int64_t n_bc = 0;
  stokes::DevBuf bc_rows, bc_ptr, bc_cols, bc_src;
  stokes::DevBuf XL_csr;          // double [nnz xl]
  stokes::DevBuf M_full, L_full;  // double [nnz p2full]
  bool strain = false;            // velocity block alpha M + mu (L + D)
  stokes::DevBuf D_full;          // double [nnz p2full][dim*dim] grad-div blocks (strain)
  stokes::DevBuf B_full;          // double [nnz bfull][dim]
  stokes::DevBuf MQ_csr, LQ_csr;  // double [nnz p1]
  stokes::DevBuf lam_full;        // double [n_p2]  Lambda_V

  // internal numbering: interior P2 nodes sorted by row length of A_II
  stokes::DevBuf int2nat;  // int32 [n_int]
  stokes::DevBuf nat2int;  // int32 [n_p2], -1 on the boundary
  std::vector<int32_t> h_int2nat, h_nat2int;

  // SELL operators used inside the iterations
  stokes::Sell sA;   // interior x interior (velocity), scalar values
  stokes::Sell sB;   // P1 x interior, dim planes
  stokes::Sell sBt;  // interior x P1, dim planes
  stokes::Sell sQ;   // P1 x P1, scalar values
  stokes::Sell sX;   // P1 x P1, B_I Lambda_V^-1 B_I^T (two-ring stencil)
  stokes::DevBuf A64, A32, MV64, MV32;       // values of A_II and M_II (SELL)
  stokes::DevBuf AD64, AD32;                 // A_II D^{-1}: column-scaled copy (first Chebyshev step)
  stokes::DevBuf AD16;                       // the same in half precision (FP32 velocity Chebyshev)
  int vel_half = 1;                          // FP32 velocity Chebyshev reads AD16
  int pmg_half = 1;                          // FP32 pressure V-cycles read the levels' half values
  int vel_bf = 1;                            // FP32 velocity Chebyshev keeps its direction q in bfloat16
  stokes::DevBuf AD16i, cdel_i8, cols_i8;    // eight-slot interleaved AD16 and sA column indices (bfloat16 steps)
  stokes::DevBuf cdel_i, cols_i;             // four-slot interleaved sA column indices (with A32i)
  stokes::DevBuf A32i;                       // four-slot interleaved A32 (FP32 velocity product of K_gamma)
  int vel_il = 1;                            // the bfloat16 Chebyshev step reads the interleaved copies
  int vel_af = 1;                            // ... and computes the columns of affine slots
  int cheb_defer = 1;                        // bfloat16 velocity Chebyshev: sum the directions in a closing step (z not carried)
  int gram_cgs2 = 1;                         // FGMRES: the CGS2 second projection from the basis Gram matrix (one pass fewer)
  int vel_pair = 1;                          // velocity slots in pair order; 1: the bfloat16 step gathers flagged pairs at once (2: order only)
  stokes::DevBuf AB64, AB32;                 // strain: [nnz_pad][dim*dim] blocks alpha M + mu (L + D)
  stokes::DevBuf B64, B32, Bt64, Bt32;       // [nnz_pad][dim]
  stokes::DevBuf MQ64, MQ32, LQ64, LQ32, XQ64, XQ32;  // XQ = M_Q + L_Q
  stokes::DevBuf dA64, dA32, dMV64, dMV32;   // inverse diagonals (interior)
  stokes::DevBuf dMQ64, dMQ32, dXQ64, dXQ32, dLQ64, dLQ32;
  stokes::DevBuf lamInv64, lamInv32;         // 1 / Lambda_V on interior nodes
  stokes::DevBuf XL64, XL32;                 // values of B_I Lambda_V^-1 B_I^T (SELL sX)
  stokes::DevBuf mQ;                         // M_Q 1 (double, n_p1)
  double mQ_sum = 0;

  stokes::Bounds bA, bMV, bMQ, bXQ, bLQ, bXQ_smooth;

  // pressure multigrid: mgq on eps M_Q + L_Q (rediscretised coarse levels,
  // level 0 is sQ / XQ); mgx on B_I Lambda_V^-1 B_I^T + M_Q with Galerkin
  // coarse levels P^T A P
  stokes::MgHier mgq, mgx;
  int mg_smooth_degree = 2, mg_coarse_degree = 24;
  int slice_yq = -1;                    // > 0: the slice schedule walks a slab's blocks per y chunk (this many per plane); -1: 8
  int slice_sched = -1;                 // > 0: interleave the row types in runs of this many slices (wide gathering kernels); -1: by size
  stokes::DevBuf rperm;                 // that schedule over the interior (velocity) rows
  int zblock = -1;                       // lattice planes per block of the interior row order (0: whole slab, -1: by size)
  int mg_es = 1;                        // pressure-MG lanes per row: 1 by level size, -1 timed, 0 one lane, 2-16 fixed
  int64_t mg_dense_max = 1500;          // largest level solved densely
  double mg_smooth_ratio = 10.0;
  int use_mgx = 1;                      // lumped CC: precondition with mgx (0: mgq)
  // P3/P2: build the Galerkin hierarchy too (0: only the eps M_Q + L_Q one),
  // its P2 pressure level smoothed on [lambda_max / mgx_p2_ratio,
  // lambda_max] at degree mgx_p2_degree
  int mgx_p3 = 1;
  double mgx_p2_ratio = 10.0;
  int mgx_p2_degree = 2;

  // velocity multigrid (built on first use; level 0 is sA / A, the coarse
  // levels rediscretise alpha M + mu L on the coarse Kuhn meshes)
  std::vector<std::unique_ptr<stokes::VmgLevel>> vmg;
  bool vmg_built = false;
  double vmg_mu = -1.0;                 // mu the hierarchy was built for
  int64_t vmg_dense_n = 0;              // rows of the coarsest level if solved densely
  stokes::DevBuf vmg_cinv64, vmg_cinv32;
  int vmg_smooth_degree = 3;

  // lanes per row of the velocity-row kernels, key W * 2 + (FP32 ? 1 : 0)
  std::map<int, int> lanes;
  int force_lanes = 0;                  // > 0: use this G everywhere (tuning, tests)

  stokes::RedScratch red;
  stokes::DevBuf scal;  // Scalars pool
  int scal_count = 0;
  std::map<std::string, stokes::DevBuf> ws;  // named workspaces (grow-only)

  stokes::DevBuf ones64, ones32;  // n_p1 * 8 ones (pressure sums)

  // timing of the dominant SpMV (opts.profile): event pairs, read at the end
  int prof_on = 0, prof_idx = 0, prof_seen = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  double prof_bytes = 0;
  double abytes = 0;  // algorithmic bytes of the kernels launched since the call began (bytes_alg)
  stokes::PhaseTimer phase[stokes::NUM_PHASES];  // phase times of stokes_solve_info (profile = 1)

  // pinned host mirror of the solver scalars
  stokes::Scalars* h_scal = nullptr;

  std::map<std::string, std::pair<void*, size_t>> ws_host;  // pinned host buffers
  uint64_t ws_gen = 1;  // bumped whenever a workspace moves (captured graphs go stale)

  // captured kernel sequences replayed with hipGraphLaunch
  struct Graph {
    hipGraphExec_t exec = nullptr;
    uint64_t gen = 0;
    int eager_runs = 0;
    double bytes = 0;  // algorithmic bytes of one replay
  };
  std::map<std::string, Graph> graphs;
  int use_graphs = 1;
  int cg_check_every = 2;  // inner CG: iterations between host convergence checks

  void* workspace(const std::string& name, size_t bytes) {
    auto& b = ws[name];
    void* old = b.p;
    b.ensure(bytes);
    if (b.p != old) ++ws_gen;
    return b.p;
  }
  // Run `enqueue` (a fixed kernel sequence on `stream`) through a cached graph.
  void run_graph(const std::string& key, const std::function<void()>& enqueue);
  void clear_graphs();
  void* workspace_host(const std::string& name, size_t bytes);
  ~stokes_ctx();
};

// Launchers for the kernels in kernels.h.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "kernels.h"
#include "ops.h"

namespace stokes {
namespace ops {

int grid_for(int64_t rows) {
  const int64_t nb = (rows + kBlock - 1) / kBlock;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nb, kMaxBlocks)));
}

// One row (group) per thread and as many workgroups as that takes (a multiple
// of 8 for the XCD partition): the dispatcher then balances rows of
// different lengths across the CUs instead of a fixed grid-stride share.
int grid_full(int64_t rows) {
  const int64_t nb = (rows + kBlock - 1) / kBlock;
  return static_cast<int>(std::max<int64_t>(8, std::min<int64_t>((nb + 7) / 8 * 8, int64_t(1) << 24)));
}

void check_launch() { HIP_CHECK(hipGetLastError()); }

template <>
const double* pick<double>(const DevBuf& b64, const DevBuf&) {
  return b64.as<double>();
}
template <>
const float* pick<float>(const DevBuf&, const DevBuf& b32) {
  return b32.as<float>();
}

// Timing of the dominant kernel (the velocity-block SpMV) with HIP events on
// the context stream; events are read back at the end of the solve.  One
// launch in kProfStride is bracketed (every launch does the same work; the
// stride is prime to the 4 steps of one polynomial, so the samples rotate
// over its positions), so the event records add little to the timed solve.
constexpr int kProfStride = 7;
bool prof_begin(stokes_ctx* c, const Sell* S, const void* vals, const void* avals) {
  if (!c->prof_on || S != &c->sA || vals != avals) return false;
  if (c->prof_seen++ % kProfStride != 0) return false;
  if (c->prof_idx >= static_cast<int>(c->prof_ev.size())) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_CHECK(hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return false;  // launches inside a graph are not timed
  HIP_CHECK(hipEventRecord(c->prof_ev[c->prof_idx].first, c->stream));
  return true;
}

void prof_end(stokes_ctx* c, double bytes) {
  HIP_CHECK(hipEventRecord(c->prof_ev[c->prof_idx].second, c->stream));
  c->prof_idx++;
  c->prof_bytes = bytes;
}

double phase_collect(stokes_ctx* c, int k) {
  PhaseTimer& t = c->phase[k];
  if (t.idx == 0) return t.acc;
  HIP_CHECK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < t.idx; ++i) {
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, t.ev[i].first, t.ev[i].second));
    t.acc += ms * 1e-3;
  }
  t.idx = 0;
  return t.acc;
}

bool phase_begin(stokes_ctx* c, int k) {
  if (c->prof_on < 2) return false;
  PhaseTimer& t = c->phase[k];
  if (t.ev.empty()) {
    t.ev.resize(1024);
    for (auto& pr : t.ev) {
      HIP_CHECK(hipEventCreate(&pr.first));
      HIP_CHECK(hipEventCreate(&pr.second));
    }
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_CHECK(hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return false;
  if (t.idx >= static_cast<int>(t.ev.size())) phase_collect(c, k);  // pool full: fold into acc
  HIP_CHECK(hipEventRecord(t.ev[t.idx].first, c->stream));
  return true;
}

void phase_end(stokes_ctx* c, int k) noexcept {
  PhaseTimer& t = c->phase[k];
  if (hipEventRecord(t.ev[t.idx].second, c->stream) == hipSuccess) t.idx++;
}

namespace {

template <int V>
using IC = std::integral_constant<int, V>;

// W in {1,2,3,4,6,8,12,16,24}
template <class F>
void dispatch_w(int W, F&& f) {
  switch (W) {
    case 1: f(IC<1>{}); break;
    case 2: f(IC<2>{}); break;
    case 3: f(IC<3>{}); break;
    case 4: f(IC<4>{}); break;
    case 6: f(IC<6>{}); break;
    case 8: f(IC<8>{}); break;
    case 12: f(IC<12>{}); break;
    case 16: f(IC<16>{}); break;
    case 24: f(IC<24>{}); break;
    default: throw Error(STOKES_ERR_UNSUPPORTED, "unsupported vector width " + std::to_string(W));
  }
}

// dim in {2,3}, nrb in {1,2,4,8}
template <class F>
void dispatch_dn(int D, int NRB, F&& f) {
  auto inner = [&](auto Dc) {
    switch (NRB) {
      case 1: f(Dc, IC<1>{}); break;
      case 2: f(Dc, IC<2>{}); break;
      case 4: f(Dc, IC<4>{}); break;
      case 8: f(Dc, IC<8>{}); break;
      default: throw Error(STOKES_ERR_UNSUPPORTED, "unsupported batch " + std::to_string(NRB));
    }
  };
  if (D == 3) inner(IC<3>{});
  else if (D == 2) inner(IC<2>{});
  else throw Error(STOKES_ERR_UNSUPPORTED, "dim");
}

inline double* partials(stokes_ctx* c) { return c->red.partials.as<double>(); }

// Lanes per row G of the velocity-row kernels: the largest of 8, 4, 2 not
// above the request that divides W (the compiled variants).
template <int WW, class F>
void with_g(int G, F&& f) {
  if constexpr (WW % 8 == 0) {
    if (G >= 8) return f(IC<8>{});
  }
  if constexpr (WW % 4 == 0) {
    if (G >= 4) return f(IC<4>{});
  }
  if constexpr (WW % 2 == 0) {
    if (G >= 2) return f(IC<2>{});
  }
  f(IC<1>{});
}

// Entry-split lanes E of a scalar operator (Sell::es, tuned per multigrid
// level); compiled for the pressure widths W in {1, 2, 4, 8}.  Returns false
// (nothing launched) for other E or W.
template <int WW, class F>
bool with_e(int E, F&& f) {
  if constexpr (WW == 1 || WW == 2 || WW == 4 || WW == 8) {
    switch (E) {
      case 2: f(IC<2>{}); return true;
      case 4: f(IC<4>{}); return true;
      case 8: f(IC<8>{}); return true;
      case 16: f(IC<16>{}); return true;
      default: return false;
    }
  } else {
    (void)E;
    (void)f;
    return false;
  }
}

// Index of the interleaved copies of the velocity pattern (iw slots per group).
SellIdx vel_il_idx(stokes_ctx* c, int W, int iw) {
  SellIdx ix = c->sA.idx(W);
  ix.cdel = (iw == 8 ? c->cdel_i8 : c->cdel_i).as<const uint8_t>();
  ix.cols = (iw == 8 ? c->cols_i8 : c->cols_i).as<const int32_t>();
  if (!c->vel_af) ix.cmeta = nullptr;  // read the packed offsets of affine slots too
  return ix;
}

// Before tuning: the largest G leaving each lane at least 3 components.
int heuristic_lanes(int W) {
  for (int g : {8, 4, 2})
    if (W % g == 0 && W / g >= 3) return g;
  return 1;
}

int lanes_w(stokes_ctx* c, int W, bool f32) {
  if (c->force_lanes > 0) return c->force_lanes;
  const auto it = c->lanes.find(W * 2 + (f32 ? 1 : 0));
  return it != c->lanes.end() ? it->second : heuristic_lanes(W);
}

// B^T rows have their own tuned G (key offset kBtKey)
constexpr int kBtKey = 1 << 20;
int lanes_bt(stokes_ctx* c, int W, bool f32) {
  if (c->force_lanes > 0) return c->force_lanes;
  const auto it = c->lanes.find(kBtKey + W * 2 + (f32 ? 1 : 0));
  return it != c->lanes.end() ? it->second : lanes_w(c, W, f32);
}

// the bfloat16-direction Chebyshev kernels too (key offset kQbKey)
constexpr int kQbKey = 2 << 20;
int lanes_qb(stokes_ctx* c, int W) {
  if (c->force_lanes > 0) return c->force_lanes;
  const auto it = c->lanes.find(kQbKey + W * 2 + 1);
  return it != c->lanes.end() ? it->second : lanes_w(c, W, true);
}

// velocity-row operators use the tuned G; the pressure operators one lane per row
int lanes_op(stokes_ctx* c, const Sell* S, int W, bool f32) {
  if (S == &c->sBt) return lanes_bt(c, W, f32);
  return S == &c->sA ? lanes_w(c, W, f32) : 1;
}

int lanes_rows(stokes_ctx* c, int64_t nrows, int W, bool f32) {
  return nrows == c->n_int ? lanes_w(c, W, f32) : 1;
}

template <int NS>
void finish(stokes_ctx* c, int64_t rows, int kind, int W, Scalars* sc, int cps, int nsys, int first, double* res) {
  hipLaunchKernelGGL((k_finish<NS>), dim3(1), dim3(kBlock), 0, c->stream, (const double*)partials(c), grid_for(rows),
                     kind, W, sc, cps, nsys, first, res);
}

template <class T> const DevBuf& bvals(stokes_ctx* c);
template <> const DevBuf& bvals<double>(stokes_ctx* c) { return c->B64; }
template <> const DevBuf& bvals<float>(stokes_ctx* c) { return c->B32; }
template <class T> const DevBuf& btvals(stokes_ctx* c);
template <> const DevBuf& btvals<double>(stokes_ctx* c) { return c->Bt64; }
template <> const DevBuf& btvals<float>(stokes_ctx* c) { return c->Bt32; }
template <class T> const DevBuf& avals(stokes_ctx* c);
template <> const DevBuf& avals<double>(stokes_ctx* c) { return c->A64; }
template <> const DevBuf& avals<float>(stokes_ctx* c) { return c->A32; }

}  // namespace

namespace {
// S = ms * (stored values); ms is folded into the product's coefficient
template <class T, class TM>
void spmv_impl(stokes_ctx* c, const Sell& S, const TM* vals, T ms, int W, const T* x, T* y, T a, const T* yin, T b) {
  const int G = lanes_op(c, &S, W, std::is_same<T, float>::value);
  bool il = false;
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    // the FP32 velocity product (K_gamma in the FGMRES cycle) on the
    // interleaved copy of A_II, G lanes per row
    if constexpr (std::is_same<T, float>::value && std::is_same<TM, float>::value) {
      if (&S == &c->sA && c->vel_il && c->A32i.p && (const void*)vals == c->A32.p) {
        with_g<WW>(G, [&](auto Gc) {
          constexpr int GG = decltype(Gc)::value;
          hipLaunchKernelGGL((k_spmv<T, WW, GG, TM, true>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0,
                             c->stream, S.nrows, vel_il_idx(c, WW, il_width<float>()), c->A32i.as<const float>(), x, y,
                             (T)(a * ms), yin, b);
        });
        il = true;
        return;
      }
    }
    if (S.es > 1 && with_e<WW>(S.es, [&](auto Ec) {
          constexpr int EE = decltype(Ec)::value;
          hipLaunchKernelGGL((k_spmv_es<T, WW, EE, TM>), dim3(grid_full(S.nrows * EE)), dim3(kBlock), 0, c->stream,
                             S.nrows, S.idx(WW), vals, x, y, (T)(a * ms), yin, b);
        }))
      return;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_spmv<T, WW, GG, TM>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream,
                         S.nrows, S.idx(WW), vals, x, y, (T)(a * ms), yin, b);
    });
  });
  check_launch();
  // operator, x gathered, y written (and yin read)
  count_bytes(c, op_bytes(S, sizeof(TM), !il || c->vel_af) + double(S.ncols) * W * sizeof(T) +
                     double(S.nrows) * W * sizeof(T) * (yin ? 2 : 1));
}
}  // namespace

template <class T>
void spmv(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* x, T* y, T a, const T* yin, T b) {
  spmv_impl<T, T>(c, S, vals, (T)1, W, x, y, a, yin, b);
}

void spmv_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* x, float* y, float a,
             const float* yin, float b) {
  spmv_impl<float, _Float16>(c, S, vals, ms, W, x, y, a, yin, b);
}

template <class T>
void Bmul(stokes_ctx* c, int nrb, const T* u, T* p, T a, const T* pin, T b) {
  const Sell& S = c->sB;
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_B<T, D, N>), dim3(grid_full(S.nrows)), dim3(kBlock), 0, c->stream, S.nrows,
                       S.idx(), bvals<T>(c).template as<T>(), u, p, a, pin, b);
  });
  check_launch();
  // B (dim planes), u gathered, p written (and pin read)
  count_bytes(c, op_bytes(S, sizeof(T)) + double(S.ncols) * c->dim * nrb * sizeof(T) +
                     double(S.nrows) * nrb * sizeof(T) * (pin ? 2 : 1));
}

template <class T>
void Btmul(stokes_ctx* c, int nrb, const T* p, const T* scale, T* u, T a, const T* uin, T b, T* btout) {
  const Sell& S = c->sBt;
  const int G = lanes_op(c, &S, c->dim * nrb, std::is_same<T, float>::value);
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    with_g<D * N>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_Bt<T, D, N, GG>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream, S.nrows,
                         S.idx(D * N), btvals<T>(c).template as<T>(), p, scale, u,
                         a, uin, b, btout);
    });
  });
  check_launch();
  // B^T (dim planes), p gathered, row scale read, u written (and uin read, btout written)
  count_bytes(c, op_bytes(S, sizeof(T)) + double(S.ncols) * nrb * sizeof(T) + (scale ? double(S.nrows) * sizeof(T) : 0) +
                     double(S.nrows) * c->dim * nrb * sizeof(T) * (1 + (uin ? 1 : 0) + (btout ? 1 : 0)));
}

template <class T> const DevBuf& abvals(stokes_ctx* c);
template <> const DevBuf& abvals<double>(stokes_ctx* c) { return c->AB64; }
template <> const DevBuf& abvals<float>(stokes_ctx* c) { return c->AB32; }

template <class T>
void velop(stokes_ctx* c, int nrb, const T* x, T* y, T a, const T* yin, T b) {
  if (!c->strain) return spmv<T>(c, c->sA, avals<T>(c).template as<T>(), c->dim * nrb, x, y, a, yin, b);
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_spmv_blk<T, D, N>), dim3(grid_full(c->n_int)), dim3(kBlock), 0, c->stream, c->n_int,
                       c->sA.idx(D * N), abvals<T>(c).template as<T>(), x, y, a, yin, b);
  });
  check_launch();
  // dim x dim blocks per entry, x gathered, y written (and yin read)
  const double W = double(c->dim) * nrb;
  count_bytes(c, double(c->sA.nnz_pad) * c->dim * c->dim * sizeof(T) + c->sA.idx_bytes_af +
                     double(c->n_int) * W * sizeof(T) * (yin ? 3 : 2));
}

template <class T>
void momentum(stokes_ctx* c, int nrb, const T* u, const T* p, const T* extra, T* y, T sgn, const T* yin) {
  if (c->strain) {
    dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
      constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
      hipLaunchKernelGGL((k_momentum_blk<T, D, N>), dim3(grid_full(c->n_int)), dim3(kBlock), 0, c->stream, c->n_int,
                         c->sA.idx(D * N), abvals<T>(c).template as<T>(), c->sBt.idx(D * N), btvals<T>(c).template as<T>(), u,
                         p, extra, y, sgn, yin);
    });
    check_launch();
    count_bytes(c, double(c->sA.nnz_pad) * c->dim * c->dim * sizeof(T) + c->sA.idx_bytes_af +
                       op_bytes(c->sBt, sizeof(T)) + double(c->n_p1) * nrb * sizeof(T) +
                       double(c->n_int) * c->dim * nrb * sizeof(T) * (2 + (extra ? 1 : 0) + (yin ? 1 : 0)));
    return;
  }
  const int G = lanes_w(c, c->dim * nrb, std::is_same<T, float>::value);
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    with_g<D * N>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_momentum<T, D, N, GG>), dim3(grid_full(c->n_int * GG)), dim3(kBlock), 0, c->stream,
                         c->n_int, c->sA.idx(D * N), avals<T>(c).template as<T>(), c->sBt.idx(D * N),
                         btvals<T>(c).template as<T>(), u, p, extra, y, sgn, yin);
    });
  });
  check_launch();
  // A and B^T, u and p gathered, y written (extra and yin read)
  count_bytes(c, op_bytes(c->sA, sizeof(T)) + op_bytes(c->sBt, sizeof(T)) + double(c->n_p1) * nrb * sizeof(T) +
                     double(c->n_int) * c->dim * nrb * sizeof(T) * (2 + (extra ? 1 : 0) + (yin ? 1 : 0)));
}

template <class T>
void dot_dev(stokes_ctx* c, int64_t nrows, int W, const T* x, const T* y, const double* rw, double* res) {
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    hipLaunchKernelGGL((k_dot<T, WW>), dim3(grid_for(nrows)), dim3(kBlock), 0, c->stream, nrows, x, y, rw, res,
                       partials(c));
    finish<WW>(c, nrows, FIN_STORE, WW, nullptr, 1, 0, 0, res);
  });
  check_launch();
  count_bytes(c, double(nrows) * (W * sizeof(T) * (y == nullptr || x == y ? 1 : 2) + (rw ? sizeof(double) : 0)));
}

template <class T>
std::vector<double> dot_host(stokes_ctx* c, int64_t nrows, int W, const T* x, const T* y, const double* rw) {
  double* res = c->red.result.as<double>();
  dot_dev<T>(c, nrows, W, x, y, rw, res);
  double* hp = static_cast<double*>(c->workspace_host("dot_h", std::max(W, kMaxSys) * sizeof(double)));
  HIP_CHECK(hipMemcpyAsync(hp, res, W * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  return std::vector<double>(hp, hp + W);
}

template <class T>
void remove_mean(stokes_ctx* c, int nrb, T* x) {
  remove_mean_into<T>(c, nrb, x, x);
}

template <class T>
void remove_mean_into(stokes_ctx* c, int nrb, const T* x, T* y) {
  const T* ones = std::is_same<T, double>::value ? (const T*)c->ones64.p : (const T*)c->ones32.p;
  const int nb = grid_for(c->n_p1);
  dispatch_w(nrb, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_dot<T, N>), dim3(nb), dim3(kBlock), 0, c->stream, c->n_p1, x, ones,
                       (const double*)nullptr, (double*)nullptr, partials(c));
    check_launch();
    hipLaunchKernelGGL((k_shift_p<T, N>), dim3(nb), dim3(kBlock), 0, c->stream, c->n_p1, x, y,
                       (const double*)partials(c), nb, 1.0 / double(c->n_p1));
  });
  check_launch();
  count_bytes(c, double(c->n_p1) * nrb * sizeof(T) * 3);  // sum pass, then read x and write y
}

template <class T>
void normalize_pressure(stokes_ctx* c, int nrb, T* x) {
  double* res = c->red.result.as<double>() + kMaxSys;
  const T* ones = std::is_same<T, double>::value ? (const T*)c->ones64.p : (const T*)c->ones32.p;
  dispatch_w(nrb, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_dot<T, N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1,
                       (const T*)x, ones, (const double*)c->mQ.as<double>(), res, partials(c));
    finish<N>(c, c->n_p1, FIN_STORE, N, nullptr, 1, 0, 0, res);
    check_launch();
    hipLaunchKernelGGL((k_shift<T, N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1, x,
                       (const double*)res, 1.0 / c->mQ_sum);
  });
  check_launch();
  count_bytes(c, double(c->n_p1) * (nrb * sizeof(T) * 3 + sizeof(double)));  // weighted sum, then shift in place
}

template <class Tin, class Tout>
void cast(stokes_ctx* c, int64_t n, const Tin* x, Tout* y) {
  hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(grid_for(n)), dim3(kBlock), 0, c->stream, n, x, y);
  check_launch();
  count_bytes(c, double(n) * (sizeof(Tin) + sizeof(Tout)));
}

template <class T>
void axpby(stokes_ctx* c, int64_t n, T a, const T* x, T b, T* y) {
  hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n)), dim3(kBlock), 0, c->stream, n, a, x, b, y);
  check_launch();
  count_bytes(c, double(n) * sizeof(T) * 3);
}

template <class T>
void axpy_sys(stokes_ctx* c, int64_t n, int W, int cps, const double* coef, double scale, const T* v, T* y) {
  hipLaunchKernelGGL((k_axpy_sys<T>), dim3(grid_for(n)), dim3(kBlock), 0, c->stream, n, W, cps, coef, scale, v, y);
  check_launch();
  count_bytes(c, double(n) * sizeof(T) * 3);
}

template <class T>
void cg_spmv(stokes_ctx* c, int64_t nrows, const Sell* S, const T* vals, int W, const T* z, const T* extra, T* q,
             T* p, Scalars* sc, int cps, int nsys) {
  const int G = S ? lanes_op(c, S, W, std::is_same<T, float>::value) : 1;
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_cg_spmv<T, WW, GG>), dim3(grid_for(nrows * GG)), dim3(kBlock), 0, c->stream, nrows,
                         S ? S->idx(WW) : SellIdx{}, vals, z,
                         extra, q, p, sc, cps, nsys, partials(c));
      finish<WW>(c, nrows * GG, FIN_ALPHA, WW, sc, cps, nsys, 0, nullptr);
    });
  });
  check_launch();
  // operator and z gathered (z streamed without one), q and p read and written (extra read)
  count_bytes(c, (S ? op_bytes(*S, sizeof(T)) + double(S->ncols) * W * sizeof(T) : 0) +
                     double(nrows) * W * sizeof(T) * (4 + (extra ? 1 : 0) + (S ? 0 : 1)));
}

template <class T>
void cg_update(stokes_ctx* c, int64_t nrows, int W, int prec, T* x, T* r, const T* p, const T* q, const T* dinv,
               T theta_inv, T* d0, T* z, Scalars* sc, int cps, int nsys) {
  const int G = lanes_rows(c, nrows, W, std::is_same<T, float>::value);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      const int nb = grid_for(nrows * GG);
      if (prec == 2) {
        hipLaunchKernelGGL((k_cg_update<T, WW, 2, GG>), dim3(nb), dim3(kBlock), 0, c->stream, nrows, x, r, p, q, dinv,
                           theta_inv, d0, z, sc, cps, nsys, partials(c));
        finish<WW>(c, nrows * GG, FIN_RR, WW, sc, cps, nsys, 0, nullptr);
      } else if (prec == 0) {
        hipLaunchKernelGGL((k_cg_update<T, WW, 0, GG>), dim3(nb), dim3(kBlock), 0, c->stream, nrows, x, r, p, q, dinv,
                           theta_inv, d0, z, sc, cps, nsys, partials(c));
        finish<WW>(c, nrows * GG, FIN_RR, WW, sc, cps, nsys, 0, nullptr);
      } else {
        hipLaunchKernelGGL((k_cg_update<T, WW, 1, GG>), dim3(nb), dim3(kBlock), 0, c->stream, nrows, x, r, p, q, dinv,
                           theta_inv, d0, z, sc, cps, nsys, partials(c));
        finish<2 * WW>(c, nrows * GG, FIN_RR_RHO, WW, sc, cps, nsys, 0, nullptr);
      }
    });
  });
  check_launch();
  // x, r read and written, p, q read; dinv; d0 and z (or z) written
  count_bytes(c, double(nrows) * (W * sizeof(T) * (6 + (prec == 0 ? 2 : prec == 1 ? 1 : 0)) +
                                  (prec == 2 ? 0 : sizeof(T))));
}

template <class T>
void cheb_init(stokes_ctx* c, int64_t nrows, int W, const T* r, const T* dinv, T theta_inv, T* d0, T* z) {
  const int G = lanes_rows(c, nrows, W, std::is_same<T, float>::value);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_cheb_init<T, WW, GG>), dim3(grid_for(nrows * GG)), dim3(kBlock), 0, c->stream, nrows, r,
                         dinv, theta_inv, d0, z);
    });
  });
  check_launch();
  count_bytes(c, double(nrows) * (W * sizeof(T) * 3 + sizeof(T)));
}

namespace {
template <class T, class TM>
void cheb_first_impl(stokes_ctx* c, const Sell& S, const TM* vals, T ms, const TM* scaled, int W, const T* r,
                     const T* dinv, T theta_inv, T* d1, T* res, T* z, T c1, T c2, int accumulate) {
  const int G = lanes_op(c, &S, W, std::is_same<T, float>::value);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    if (!scaled && S.es > 1 && with_e<WW>(S.es, [&](auto Ec) {
          constexpr int EE = decltype(Ec)::value;
          auto kern = accumulate ? k_cheb_first_es<T, WW, 1, EE, TM> : k_cheb_first_es<T, WW, 0, EE, TM>;
          hipLaunchKernelGGL(kern, dim3(grid_full(S.nrows * EE)), dim3(kBlock), 0, c->stream, S.nrows, S.idx(WW), vals,
                             ms, r, dinv, theta_inv, d1, res, z, c1, c2);
        }))
      return;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      const int nb = grid_full(S.nrows * GG);
      auto go = [&](auto kern, const TM* v) {
        hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, c->stream, S.nrows, S.idx(WW), v, ms, r, dinv, theta_inv,
                           d1, res, z, c1, c2);
      };
      if (scaled) {
        if (accumulate) go(k_cheb_first<T, WW, 1, GG, 1, TM>, scaled);
        else go(k_cheb_first<T, WW, 0, GG, 1, TM>, scaled);
      } else {
        if (accumulate) go(k_cheb_first<T, WW, 1, GG, 0, TM>, vals);
        else go(k_cheb_first<T, WW, 0, GG, 0, TM>, vals);
      }
    });
  });
  check_launch();
  // operator, r gathered (and dinv with the unscaled one), dinv read; res, d1, z written (z read)
  count_bytes(c, op_bytes(S, sizeof(TM)) + double(S.ncols) * (W * sizeof(T) + (scaled ? 0 : sizeof(T))) +
                     double(S.nrows) * (sizeof(T) + W * sizeof(T) * (3 + (accumulate ? 1 : 0))));
}
}  // namespace

template <class T>
void cheb_first(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* r, const T* dinv, T theta_inv, T* d1,
                T* res, T* z, T c1, T c2, int accumulate) {
  // the velocity operator has a column-scaled copy S D^{-1}
  const T* scaled = (&S == &c->sA && vals == avals<T>(c).template as<T>()) ? pick<T>(c->AD64, c->AD32) : nullptr;
  cheb_first_impl<T, T>(c, S, vals, (T)1, scaled, W, r, dinv, theta_inv, d1, res, z, c1, c2, accumulate);
}

void cheb_first_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* r,
                   const float* dinv, float theta_inv, float* d1, float* res, float* z, float c1, float c2,
                   int accumulate) {
  cheb_first_impl<float, _Float16>(c, S, vals, ms, nullptr, W, r, dinv, theta_inv, d1, res, z, c1, c2, accumulate);
}

void cheb_first_h(stokes_ctx* c, int W, const float* r, const float* dinv, float theta_inv, float* q1, float* res,
                  float* z, float c1, float c2) {
  const Sell& S = c->sA;
  const int G = lanes_op(c, &S, W, true);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_cheb_first_q<float, _Float16, WW, 0, GG, 8>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0,
                         c->stream, S.nrows, S.idx(WW),
                         (const _Float16*)c->AD16.as<_Float16>(), r, dinv, theta_inv, q1, res, z, c1, c2);
    });
  });
  check_launch();
  // half values, r gathered, dinv read; q1, res, z written
  count_bytes(c, op_bytes(S, 2) + double(S.nrows) * 4.0 * (4.0 * W + 1.0));
}

void cheb_first_hb(stokes_ctx* c, int W, const float* r, const float* dinv, float theta_inv, uint16_t* q1,
                   float* res, float* z, float c1, float c2, bool zw) {
  const Sell& S = c->sA;
  const int G = lanes_qb(c, W);
  int wp = W;
  bool il = false;
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    wp = bf_width<WW>();
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      if (c->vel_il && c->AD16i.p) {  // the eight-slot interleaved copies
        auto kern = zw ? k_cheb_first_qb<_Float16, WW, 0, GG, 8, true> : k_cheb_first_qb<_Float16, WW, 2, GG, 8, true>;
        hipLaunchKernelGGL(kern, dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream, S.nrows,
                           vel_il_idx(c, WW, il_width<_Float16>()),
                           (const _Float16*)c->AD16i.as<_Float16>(), r, dinv, theta_inv, q1, res, z, c1, c2);
        il = true;
        return;
      }
      auto kern = zw ? k_cheb_first_qb<_Float16, WW, 0, GG> : k_cheb_first_qb<_Float16, WW, 2, GG>;
      hipLaunchKernelGGL(kern, dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream, S.nrows, S.idx(WW),
                         (const _Float16*)c->AD16.as<_Float16>(), r, dinv, theta_inv, q1, res, z, c1, c2);
    });
  });
  check_launch();
  // half values, r gathered; res (floats) and q1 (bfloat16) written; dinv
  // read and z written unless deferred
  count_bytes(c, op_bytes(S, 2, !il || c->vel_af) +
                     double(S.nrows) * (4.0 * (2.0 * W) + 2.0 * wp + (zw ? 4.0 * (W + 1.0) : 0.0)));
}

void cheb_step_hb(stokes_ctx* c, int W, const uint16_t* q, uint16_t* qn, const float* res_in, float* res_out,
                  float* z, const float* dinv, float c1, float c2, const QSum* fin, bool zw) {
  const Sell& S = c->sA;
  // the timed launches: the steps that carry the iterate (deferred or not), not the closing one
  const bool timed = fin == nullptr && prof_begin(c, &S, nullptr, nullptr);
  const int zm = fin ? 2 : zw ? 0 : 1;
  QSum fa{};
  if (fin) {
    if (fin->n < 0 || fin->n > kQSumMax) throw Error(STOKES_ERR_ARG, "deferred Chebyshev sum too long");
    fa = *fin;
  }
  const int G = lanes_qb(c, W);
  int wp = W;
  bool il = false;
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    wp = bf_width<WW>();
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      const int nb = grid_full(S.nrows * GG);
      if constexpr (BfRaw<bf_width<WW>(), WW / GG>::kOn) {
        if (c->vel_il && c->AD16i.p) {  // the eight-slot interleaved copies
          auto kern = zm == 0   ? k_cheb_step_qb<_Float16, WW, GG, 8, true, 0>
                      : zm == 1 ? k_cheb_step_qb<_Float16, WW, GG, 8, true, 1>
                                : k_cheb_step_qb<_Float16, WW, GG, 8, true, 2>;
          hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, c->stream, S.nrows, vel_il_idx(c, WW, il_width<_Float16>()),
                             (const _Float16*)c->AD16i.as<_Float16>(), q, qn, res_in, res_out, z, dinv, c1, c2, fa);
          il = true;
          return;
        }
      }
      auto kern = zm == 0   ? k_cheb_step_qb<_Float16, WW, GG, 8, false, 0>
                  : zm == 1 ? k_cheb_step_qb<_Float16, WW, GG, 8, false, 1>
                            : k_cheb_step_qb<_Float16, WW, GG, 8, false, 2>;
      hipLaunchKernelGGL(kern, dim3(nb), dim3(kBlock), 0, c->stream, S.nrows, S.idx(WW),
                         (const _Float16*)c->AD16.as<_Float16>(), q, qn, res_in, res_out, z, dinv, c1, c2, fa);
    });
  });
  check_launch();
  // algorithmic bytes: the stored operator once (half values of every padded
  // entry, the column-index structure it reads: slot words alone for the
  // affine slices of the interleaved copy); q read once (gathered and own
  // row, WP bfloat16); res_in read (W floats); then
  //   carrying z:  res_out and z written, z and dinv read, qn written;
  //   deferred:    res_out and qn written;
  //   closing:     r and the n earlier directions read, dinv read, z written
  const double vec = zm == 0   ? 4.0 * (W * 4.0 + 1.0) + 2.0 * 2.0 * wp
                     : zm == 1 ? 4.0 * (W * 2.0) + 2.0 * 2.0 * wp
                               : 4.0 * (W * 3.0 + 1.0) + 2.0 * wp * (1.0 + fa.n);
  const double bytes = op_bytes(S, 2, !il || c->vel_af) + double(S.nrows) * vec;
  count_bytes(c, bytes);
  if (timed) prof_end(c, bytes);
}

void cheb_step_h(stokes_ctx* c, int W, const float* q, float* qn, const float* res_in, float* res_out, float* z,
                 const float* dinv, float c1, float c2) {
  const Sell& S = c->sA;
  const bool timed = prof_begin(c, &S, nullptr, nullptr);
  const int G = lanes_op(c, &S, W, true);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream, S.nrows, S.idx(WW),
                           (const _Float16*)c->AD16.as<_Float16>(), q, qn, res_in, res_out, z, dinv, c1, c2);
      };
      go(k_cheb_step_q<float, _Float16, WW, GG, 8>);
    });
  });
  check_launch();
  // algorithmic bytes: the stored operator once (half values of every padded
  // entry, the column-index structure); q gathered once; res_in, q, z read;
  // res_out, qn, z written (W floats each); dinv read
  const double bytes = op_bytes(S, 2) + double(S.nrows) * 4.0 * (W * 6.0 + 1.0);
  count_bytes(c, bytes);
  if (timed) prof_end(c, bytes);
}

void cheb_step_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* d, float* dn,
                  const float* res_in, float* res_out, float* z, const float* dinv, float c1, float c2) {
  const int G = lanes_op(c, &S, W, true);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    if (S.es > 1 && with_e<WW>(S.es, [&](auto Ec) {
          constexpr int EE = decltype(Ec)::value;
          hipLaunchKernelGGL((k_cheb_step_es<float, WW, EE, _Float16>), dim3(grid_full(S.nrows * EE)), dim3(kBlock),
                             0, c->stream, S.nrows, S.idx(WW), vals, ms, d, dn, res_in, res_out, z, dinv, c1, c2);
        }))
      return;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      hipLaunchKernelGGL((k_cheb_step<float, WW, 0, GG, _Float16>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0,
                         c->stream, S.nrows, S.idx(WW), vals, ms, d, dn, res_in, res_out, z, dinv, c1, c2,
                         (const float*)nullptr, (Scalars*)nullptr, 1, 0, 0, partials(c));
    });
  });
  check_launch();
  // half values, d gathered; res_in, z, dinv read; res_out, dn, z written
  count_bytes(c, op_bytes(S, 2) + double(S.ncols) * W * 4.0 + double(S.nrows) * 4.0 * (W * 5.0 + 1.0));
}

template <class T>
void cheb_step(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* d, T* dn, const T* res_in, T* res_out,
               T* z, const T* dinv, T c1, T c2, const T* rvec, Scalars* sc, int cps, int nsys, int first) {
  // the timed kernel is the plain Chebyshev step (no fused dot) on the velocity block
  const bool timed = rvec == nullptr && prof_begin(c, &S, (const void*)vals, (const void*)avals<T>(c).template as<T>());
  const int G = lanes_op(c, &S, W, std::is_same<T, float>::value);
  dispatch_w(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    if (!rvec && S.es > 1 && with_e<WW>(S.es, [&](auto Ec) {
          constexpr int EE = decltype(Ec)::value;
          hipLaunchKernelGGL((k_cheb_step_es<T, WW, EE>), dim3(grid_full(S.nrows * EE)), dim3(kBlock), 0, c->stream,
                             S.nrows, S.idx(WW), vals, (T)1, d, dn, res_in, res_out, z, dinv, c1, c2);
        }))
      return;
    with_g<WW>(G, [&](auto Gc) {
      constexpr int GG = decltype(Gc)::value;
      const int nb = grid_for(S.nrows * GG);
      if (rvec) {
        hipLaunchKernelGGL((k_cheb_step<T, WW, 1, GG>), dim3(nb), dim3(kBlock), 0, c->stream, S.nrows,
                           S.idx(WW), vals, (T)1, d, dn, res_in, res_out, z, dinv, c1,
                           c2, rvec, sc, cps, nsys, first, partials(c));
        finish<WW>(c, S.nrows * GG, FIN_RHO, WW, sc, cps, nsys, first, nullptr);
      } else
        hipLaunchKernelGGL((k_cheb_step<T, WW, 0, GG>), dim3(grid_full(S.nrows * GG)), dim3(kBlock), 0, c->stream, S.nrows,
                           S.idx(WW), vals, (T)1, d, dn, res_in, res_out, z, dinv, c1,
                           c2, rvec, sc, cps, nsys, first, partials(c));
    });
  });
  check_launch();
  // algorithmic bytes: the stored operator once (values of every padded
  // entry, the column-index structure); d gathered once; res_in, z, dinv
  // (and rvec) read; res_out, dn, z written
  const double bytes = op_bytes(S, sizeof(T)) + double(S.ncols) * W * sizeof(T) +
                       double(S.nrows) * sizeof(T) * (W * (rvec ? 6.0 : 5.0) + 1.0);
  count_bytes(c, bytes);
  if (timed) prof_end(c, bytes);
}

// Tuning cache (STOKES_TUNE_CACHE = path of a text file): one line
// "<problem> <lanes key> <G>" per tuned choice, where <problem> names the
// mesh, element pair, form and device.  A context whose problem is in the
// file takes its choices from there instead of timing them again.
std::string tune_problem(stokes_ctx* c) {
  hipDeviceProp_t pr;
  HIP_CHECK(hipGetDeviceProperties(&pr, c->device));
  std::string arch(pr.gcnArchName);
  for (char& ch : arch)
    if (ch == ' ' || ch == ':') ch = '_';
  char b[256];
  std::snprintf(b, sizeof(b), "d%d_n%d_p%d_s%d_rows%lld_%s", c->dim, c->mesh.n, c->mesh.order, c->strain ? 1 : 0,
                (long long)c->n_int, arch.c_str());
  return b;
}

// Fill c->lanes from the cache file; true if `key` was found.
bool tune_cache_load(stokes_ctx* c, int key) {
  const char* path = std::getenv("STOKES_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* fh = std::fopen(path, "r");
  if (!fh) return false;
  const std::string prob = tune_problem(c);
  char name[256];
  int k = 0, g = 0;
  bool found = false;
  while (std::fscanf(fh, "%255s %d %d", name, &k, &g) == 3)
    if (prob == name && (g == 1 || g == 2 || g == 4 || g == 8)) {
      c->lanes[k] = g;
      found = found || k == key;
    }
  std::fclose(fh);
  return found;
}

void tune_cache_store(stokes_ctx* c, const std::vector<int>& keys) {
  const char* path = std::getenv("STOKES_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* fh = std::fopen(path, "a");
  if (!fh) return;  // an unwritable cache only costs the timing next time
  const std::string prob = tune_problem(c);
  for (int k : keys)
    if (c->lanes.count(k)) std::fprintf(fh, "%s %d %d\n", prob.c_str(), k, c->lanes[k]);
  std::fclose(fh);
}

// Autotune G for the velocity-row kernels of width W in precision T: time the
// plain SELL product on the velocity block for every compiled G and keep the
// fastest (cached per context and, with STOKES_TUNE_CACHE, in a file;
// skipped while a graph is being captured).
template <class T>
void tune_lanes(stokes_ctx* c, int W) {
  const int key = W * 2 + (std::is_same<T, float>::value ? 1 : 0);
  if (c->force_lanes > 0 || c->lanes.count(key)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_CHECK(hipStreamIsCapturing(c->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return;
  std::vector<int> cand;
  for (int g : {1, 2, 4, 8})
    if (W % g == 0) cand.push_back(g);
  if (cand.size() == 1) {
    c->lanes[key] = 1;
    return;
  }
  if (tune_cache_load(c, key)) return;
  const int64_t n = c->n_int * W;
  DevBuf x, y;
  x.alloc(n * sizeof(T));
  y.alloc(n * sizeof(T));
  HIP_CHECK(hipMemsetAsync(x.p, 0, n * sizeof(T), c->stream));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  const Sell& S = c->sA;
  const T* vals = pick<T>(c->A64, c->A32);
  int best = cand[0];
  float best_ms = 1e30f;
  for (int g : cand) {
    c->force_lanes = g;
    spmv<T>(c, S, vals, W, x.as<T>(), y.as<T>(), T(1), nullptr, T(0));  // warm-up
    HIP_CHECK(hipEventRecord(e0, c->stream));
    for (int rep = 0; rep < 3; ++rep) spmv<T>(c, S, vals, W, x.as<T>(), y.as<T>(), T(1), nullptr, T(0));
    HIP_CHECK(hipEventRecord(e1, c->stream));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (const char* e = std::getenv("STOKES_LOG"); e && std::atoi(e) >= 1)
      std::fprintf(stderr, "[stokes] lanes W=%d %s G=%d: %.1f us per SpMV\n", W,
                   std::is_same<T, float>::value ? "fp32" : "fp64", g, 1e3 * ms / 3);
    if (ms < best_ms) {
      best_ms = ms;
      best = g;
    }
  }
  c->lanes[key] = best;
  // the same for the B^T product (pressure gathers, d value planes)
  if (W % c->dim == 0) {
    const int nrb = W / c->dim;
    DevBuf pz;
    pz.alloc(c->n_p1 * nrb * sizeof(T));
    HIP_CHECK(hipMemsetAsync(pz.p, 0, c->n_p1 * nrb * sizeof(T), c->stream));
    int bbest = best;
    float bms = 1e30f;
    for (int g : cand) {
      c->force_lanes = g;
      Btmul<T>(c, nrb, pz.as<T>(), nullptr, y.as<T>(), T(1), nullptr, T(0));  // warm-up
      HIP_CHECK(hipEventRecord(e0, c->stream));
      for (int rep = 0; rep < 3; ++rep) Btmul<T>(c, nrb, pz.as<T>(), nullptr, y.as<T>(), T(1), nullptr, T(0));
      HIP_CHECK(hipEventRecord(e1, c->stream));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (const char* e = std::getenv("STOKES_LOG"); e && std::atoi(e) >= 1)
        std::fprintf(stderr, "[stokes] lanes W=%d %s G=%d: %.1f us per B^T product\n", W,
                     std::is_same<T, float>::value ? "fp32" : "fp64", g, 1e3 * ms / 3);
      if (ms < bms) {
        bms = ms;
        bbest = g;
      }
    }
    c->lanes[kBtKey + key] = bbest;
  }
  // the bfloat16-direction Chebyshev step (FP32 contexts with the half copy)
  if (std::is_same<T, float>::value && c->AD16.p) {
    DevBuf qa, qb;
    qa.alloc(c->n_int * W * sizeof(uint16_t) * 2);
    qb.alloc(c->n_int * W * sizeof(uint16_t) * 2);
    HIP_CHECK(hipMemsetAsync(qa.p, 0, qa.bytes, c->stream));
    int qbest = best;
    float qms = 1e30f;
    const bool prof = c->prof_on;
    c->prof_on = false;
    for (int g : cand) {
      c->force_lanes = g;
      float* xr = reinterpret_cast<float*>(x.p);
      float* yz = reinterpret_cast<float*>(y.p);
      const float* di = c->dA32.as<float>();
      cheb_step_hb(c, W, qa.as<uint16_t>(), qb.as<uint16_t>(), xr, xr, yz, di, 0.5f, 0.5f, nullptr, false);  // warm-up
      HIP_CHECK(hipEventRecord(e0, c->stream));
      for (int rep = 0; rep < 3; ++rep)
        cheb_step_hb(c, W, qa.as<uint16_t>(), qb.as<uint16_t>(), xr, xr, yz, di, 0.5f, 0.5f, nullptr, false);
      HIP_CHECK(hipEventRecord(e1, c->stream));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (const char* e = std::getenv("STOKES_LOG"); e && std::atoi(e) >= 1)
        std::fprintf(stderr, "[stokes] lanes W=%d G=%d: %.1f us per bfloat16 Chebyshev step\n", W, g, 1e3 * ms / 3);
      if (ms < qms) {
        qms = ms;
        qbest = g;
      }
    }
    c->prof_on = prof;
    c->lanes[kQbKey + key] = qbest;
  }
  c->force_lanes = 0;
  tune_cache_store(c, {key, kBtKey + key, kQbKey + key});
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
  HIP_CHECK(hipStreamSynchronize(c->stream));
}

void ensure_lanes(stokes_ctx* c, int W, bool f32) {
  if (f32) tune_lanes<float>(c, W);
  else tune_lanes<double>(c, W);
}

template <class T>
void vel_in(stokes_ctx* c, int nrb, const double* src, T* dst) {
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_vel_in<T, D, N>), dim3(grid_for(c->n_int)), dim3(kBlock), 0, c->stream, c->n_int, c->n_p2,
                       c->int2nat.as<int32_t>(), src, dst);
  });
  check_launch();
  count_bytes(c, double(c->n_int) * (4.0 + c->dim * nrb * (8.0 + sizeof(T))));
}

template <class T>
void vel_out(stokes_ctx* c, int nrb, const T* src, const double* ubc, double* dst, int bnd_fill) {
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_vel_out<T, D, N>), dim3(grid_for(c->n_p2)), dim3(kBlock), 0, c->stream, c->n_p2,
                       c->nat2int.as<int32_t>(), src, ubc, dst, bnd_fill);
  });
  check_launch();
  count_bytes(c, double(c->n_p2) * 4.0 + double(c->dim) * nrb * (c->n_int * sizeof(T) + c->n_p2 * 8.0) +
                     (ubc ? double(c->n_p2 - c->n_int) * c->dim * nrb * 8.0 : 0));
}

template <class T>
void p_in(stokes_ctx* c, int nrb, const double* src, T* dst) {
  dispatch_w(nrb, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_p_in<T, N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1, src, dst);
  });
  check_launch();
  count_bytes(c, double(c->n_p1) * nrb * (8.0 + sizeof(T)));
}

template <class T>
void p_out(stokes_ctx* c, int nrb, const T* src, double* dst) {
  dispatch_w(nrb, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_p_out<T, N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1, src, dst);
  });
  check_launch();
  count_bytes(c, double(c->n_p1) * nrb * (8.0 + sizeof(T)));
}

void rhs(stokes_ctx* c, int nrb, const double* f, const double* ubc, double* F, double* g, double* fI) {
  // F~ = (M_V f)_I - A_{I,Gamma} G: interior columns by the sliced-ELL mass
  // product on f_I, boundary columns on the rows that touch the boundary
  const int W = c->dim * nrb;
  if (f) {
    if (!fI) fI = static_cast<double*>(c->workspace("rhs_fI", c->n_int * W * sizeof(double)));
    vel_in<double>(c, nrb, f, fI);
    spmv<double>(c, c->sA, c->MV64.as<double>(), W, fI, F, 1.0, nullptr, 0.0);
  } else {
    hipLaunchKernelGGL((k_set<double>), dim3(grid_for(c->n_int * W)), dim3(kBlock), 0, c->stream, c->n_int * W, 0.0,
                       F);
    count_bytes(c, double(c->n_int) * W * 8.0);
  }
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    if (c->n_bc > 0 && (f || ubc))
      hipLaunchKernelGGL((k_rhs_bnd<D, N>), dim3(grid_for(c->n_bc * kRhsLanes)), dim3(kBlock), 0, c->stream, c->n_bc,
                         c->n_p2,
                         c->bc_rows.as<int32_t>(), c->bc_ptr.as<int32_t>(), c->bc_cols.as<int32_t>(),
                         c->bc_src.as<int32_t>(), c->M_full.as<double>(), c->L_full.as<double>(),
                         c->strain ? c->D_full.as<double>() : nullptr, c->prob.alpha, c->prob.mu, f, ubc, F);
    check_launch();
    hipLaunchKernelGGL((k_rhs_p<D, N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1, c->n_p2,
                       c->nat2int.as<int32_t>(), c->bfull.rowptr.as<int32_t>(), c->bfull.cols.as<int32_t>(),
                       c->B_full.as<double>(), ubc, g);
  });
  check_launch();
  // boundary rows: their column lists and M, L (D) entries, f and ubc gathered, F rows read and written;
  // pressure rows: the full B pattern and values, ubc gathered, g written
  const double nbe = double(c->bc_cols.bytes) / 4.0, nb = double(c->bfull.nnz);
  if (c->n_bc > 0 && (f || ubc))
    count_bytes(c, nbe * (4.0 + 4.0 + 16.0 + (c->strain ? 8.0 * c->dim * c->dim : 0)) + double(c->n_bc) * (8.0 + 16.0 * W) +
                       ((f ? 1 : 0) + (ubc ? 1 : 0)) * double(c->n_p2) * W * 8.0);
  count_bytes(c, double(c->n_p1) * 4.0 + nb * (4.0 + 8.0 * c->dim) + (ubc ? double(c->n_p2) * W * 8.0 : 0) +
                     double(c->n_p1) * nrb * 8.0);
}

void adj_jp(stokes_ctx* c, int nrb, double* g) {
  double* sum = c->red.result.as<double>() + 3 * kMaxSys;
  dot_dev<double>(c, c->n_p1, nrb, g, c->ones64.as<double>(), nullptr, sum);
  dispatch_w(nrb, [&](auto Nc) {
    constexpr int N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_adj_jp<N>), dim3(grid_for(c->n_p1)), dim3(kBlock), 0, c->stream, c->n_p1,
                       c->mQ.as<double>(), (const double*)sum, 1.0 / c->mQ_sum, g);
  });
  check_launch();
  count_bytes(c, double(c->n_p1) * (8.0 + 16.0 * nrb));
}

void adj_dJdf(stokes_ctx* c, int nrb, const double* lam, double* out) {
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_adj_dJdf<D, N>), dim3(grid_for(c->n_p2)), dim3(kBlock), 0, c->stream, c->n_p2,
                       c->nat2int.as<int32_t>(), c->p2full.rowptr.as<int32_t>(), c->p2full.cols.as<int32_t>(),
                       c->M_full.as<double>(), lam, out);
  });
  check_launch();
  const double W = double(c->dim) * nrb;
  count_bytes(c, double(c->n_p2) * (8.0 + W * 8.0) + double(c->p2full.nnz) * 12.0 + double(c->n_int) * W * 8.0);
}

void adj_dJdmu(stokes_ctx* c, int nrb, const double* u_full, const double* lam, double* res_dev) {
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_adj_dJdmu<D, N>), dim3(grid_for(c->n_int)), dim3(kBlock), 0, c->stream, c->n_int, c->n_p2,
                       c->int2nat.as<int32_t>(), c->p2full.rowptr.as<int32_t>(), c->p2full.cols.as<int32_t>(),
                       c->L_full.as<double>(), c->strain ? c->D_full.as<double>() : nullptr, u_full, lam, res_dev,
                       partials(c));
    finish<N>(c, c->n_int, FIN_STORE, N, nullptr, 1, 0, 0, res_dev);
  });
  check_launch();
  const double W = double(c->dim) * nrb;
  count_bytes(c, double(c->n_int) * (12.0 + W * 8.0) + double(c->p2full.nnz) * (12.0 + (c->strain ? 8.0 * c->dim * c->dim : 0)) +
                     double(c->n_p2) * W * 8.0);
}

#define INST(T)                                                                                                      \
  template void spmv<T>(stokes_ctx*, const Sell&, const T*, int, const T*, T*, T, const T*, T);                     \
  template void Bmul<T>(stokes_ctx*, int, const T*, T*, T, const T*, T);                                            \
  template void Btmul<T>(stokes_ctx*, int, const T*, const T*, T*, T, const T*, T, T*);                             \
  template void momentum<T>(stokes_ctx*, int, const T*, const T*, const T*, T*, T, const T*);                       \
  template void velop<T>(stokes_ctx*, int, const T*, T*, T, const T*, T);                                           \
  template void dot_dev<T>(stokes_ctx*, int64_t, int, const T*, const T*, const double*, double*);                  \
  template std::vector<double> dot_host<T>(stokes_ctx*, int64_t, int, const T*, const T*, const double*);           \
  template void remove_mean<T>(stokes_ctx*, int, T*);                                                               \
  template void remove_mean_into<T>(stokes_ctx*, int, const T*, T*);                                                \
  template void normalize_pressure<T>(stokes_ctx*, int, T*);                                                        \
  template void axpby<T>(stokes_ctx*, int64_t, T, const T*, T, T*);                                                 \
  template void axpy_sys<T>(stokes_ctx*, int64_t, int, int, const double*, double, const T*, T*);                   \
  template void cg_spmv<T>(stokes_ctx*, int64_t, const Sell*, const T*, int, const T*, const T*, T*, T*, Scalars*, int, \
                           int);                                                                                 \
  template void cg_update<T>(stokes_ctx*, int64_t, int, int, T*, T*, const T*, const T*, const T*, T, T*, T*,       \
                             Scalars*, int, int);                                                                    \
  template void cheb_init<T>(stokes_ctx*, int64_t, int, const T*, const T*, T, T*, T*);                             \
  template void cheb_first<T>(stokes_ctx*, const Sell&, const T*, int, const T*, const T*, T, T*, T*, T*, T, T, int); \
  template void cheb_step<T>(stokes_ctx*, const Sell&, const T*, int, const T*, T*, const T*, T*, T*, const T*, T,  \
                             T, const T*, Scalars*, int, int, int);                                                  \
  template void vel_in<T>(stokes_ctx*, int, const double*, T*);                                                     \
  template void vel_out<T>(stokes_ctx*, int, const T*, const double*, double*, int);                                \
  template void p_in<T>(stokes_ctx*, int, const double*, T*);                                                       \
  template void p_out<T>(stokes_ctx*, int, const T*, double*);

INST(double)
INST(float)
template void cast<double, float>(stokes_ctx*, int64_t, const double*, float*);
template void cast<float, double>(stokes_ctx*, int64_t, const float*, double*);

}  // namespace ops
}  // namespace stokes

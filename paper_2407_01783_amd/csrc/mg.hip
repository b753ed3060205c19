// Geometric multigrid V-cycle for the P1 pressure operator eps M_Q + L_Q
// (eps = 1), the operator the paper uses to precondition the Schur-complement
// approximations B M^{-1} B^T / B Lambda^{-1} B^T (Sec. 4.2).  The paper
// applies two algebraic-multigrid V-cycles (Table 1, BoomerAMG); on the
// structured Kuhn mesh a geometric hierarchy is available instead:
//
//   * level l+1 has n / 2^(l+1) cells per side; its vertices are the level-0
//     vertices whose grid indices are multiples of 2^(l+1) (jittered
//     positions kept), its simplices the Kuhn split of the coarse grid, and
//     its operator M_Q + L_Q is re-assembled on that mesh;
//   * a level-l vertex with grid index f is the midpoint of the coarse Kuhn
//     edge (f - s, f + s) with s = f mod 2 (componentwise), so P1
//     interpolation averages those two coarse values; restriction is its
//     transpose;
//   * smoothing: Chebyshev-Jacobi on the upper part of each level's spectrum,
//     the same polynomial before and after the coarse correction, so the
//     cycle is symmetric and can precondition CG;
//   * coarsest level: an exact dense inverse when it has at most 1500
//     vertices, else a Chebyshev polynomial over its whole spectrum.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <memory>
#include <type_traits>

#include "kernels.h"
#include "ops.h"

namespace stokes {

namespace {

template <int V>
using IC = std::integral_constant<int, V>;

template <class F>
void dispatch_dn(int D, int NRB, F&& f) {
  auto inner = [&](auto Dc) {
    switch (NRB) {
      case 1: f(Dc, IC<1>{}); break;
      case 2: f(Dc, IC<2>{}); break;
      case 4: f(Dc, IC<4>{}); break;
      case 8: f(Dc, IC<8>{}); break;
      default: throw Error(STOKES_ERR_UNSUPPORTED, "batch");
    }
  };
  if (D == 3) inner(IC<3>{});
  else inner(IC<2>{});
}

// restriction: coarse vertex C gathers fine vertices 2C (weight 1) and
// 2C + s, 2C - s (weight 1/2) for every nonzero s in {0,1}^D
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_restrict(int nf, int nc, const T* __restrict__ rf, T* __restrict__ rc) {
  const int64_t ncv = (int64_t)ipow_dev(nc + 1, D);
  GRID_STRIDE_ROWS(C, ncv) {
    int cg[3] = {0, 0, 0};
    int64_t rem = C;
    for (int d = 0; d < D; ++d) {
      cg[d] = (int)(rem % (nc + 1));
      rem /= (nc + 1);
    }
    T acc[NRB];
    auto fid = [&](const int* g) {
      int64_t id = 0, st = 1;
      for (int d = 0; d < D; ++d, st *= (nf + 1)) id += g[d] * st;
      return id;
    };
    {
      int g[3];
      for (int d = 0; d < D; ++d) g[d] = 2 * cg[d];
      const int64_t f = fid(g);
#pragma unroll
      for (int r = 0; r < NRB; ++r) acc[r] = rf[f * NRB + r];
    }
    for (int s = 1; s < (1 << D); ++s) {
      for (int sg = -1; sg <= 1; sg += 2) {
        int g[3];
        bool ok = true;
        for (int d = 0; d < D; ++d) {
          g[d] = 2 * cg[d] + sg * ((s >> d) & 1);
          ok = ok && g[d] >= 0 && g[d] <= nf;
        }
        if (!ok) continue;
        const int64_t f = fid(g);
#pragma unroll
        for (int r = 0; r < NRB; ++r) acc[r] += T(0.5) * rf[f * NRB + r];
      }
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r) rc[C * NRB + r] = acc[r];
  }
}

// interpolation, added to the fine vector: ef[f] += (ec[(f-s)/2] + ec[(f+s)/2]) / 2
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_prolong_add(int nf, int nc, const T* __restrict__ ec, T* __restrict__ ef) {
  const int64_t nfv = (int64_t)ipow_dev(nf + 1, D);
  GRID_STRIDE_ROWS(f, nfv) {
    int fg[3] = {0, 0, 0};
    int64_t rem = f;
    for (int d = 0; d < D; ++d) {
      fg[d] = (int)(rem % (nf + 1));
      rem /= (nf + 1);
    }
    int64_t a = 0, b = 0, st = 1;
    for (int d = 0; d < D; ++d, st *= (nc + 1)) {
      const int s = fg[d] & 1;
      a += ((fg[d] - s) / 2) * st;
      b += ((fg[d] + s) / 2) * st;
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r) ef[f * NRB + r] += T(0.5) * (ec[a * NRB + r] + ec[b * NRB + r]);
  }
}

// y[i][r] = sum_j Cinv[i][j] x[j][r]   (coarsest-level solve): one wavefront
// per row, coalesced over j, wavefront-shuffle reduction
template <typename T, int NRB>
__global__ __launch_bounds__(kBlock) void k_dense_mv(int64_t n, const T* __restrict__ Ci, const T* __restrict__ x,
                                                     T* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= n) return;  // whole wavefronts exit together
  double acc[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) acc[r] = 0;
  for (int64_t j = lane; j < n; j += 64) {
    const double a = Ci[row * n + j];
#pragma unroll
    for (int r = 0; r < NRB; ++r) acc[r] += a * (double)x[j * NRB + r];
  }
#pragma unroll
  for (int r = 0; r < NRB; ++r) acc[r] = wave_sum(acc[r]);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < NRB; ++r) y[row * NRB + r] = (T)acc[r];
}

// Inverse of a small SPD matrix by Cholesky (host).
std::vector<double> spd_inverse(std::vector<double> A, int64_t n) {
  for (int64_t j = 0; j < n; ++j) {  // A = L L^T in place (lower)
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0)) throw Error(STOKES_ERR_BREAKDOWN, "coarsest multigrid operator is not positive definite");
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
  }
  std::vector<double> inv(n * n, 0.0), col(n);
  for (int64_t c = 0; c < n; ++c) {  // solve L L^T x = e_c
    for (int64_t i = 0; i < n; ++i) {
      double s = i == c ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) s -= A[i * n + k] * col[k];
      col[i] = s / A[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = col[i];
      for (int64_t k = i + 1; k < n; ++k) s -= A[k * n + i] * col[k];
      col[i] = s / A[i * n + i];
    }
    for (int64_t i = 0; i < n; ++i) inv[i * n + c] = col[i];
  }
  return inv;
}

struct Cheb {
  double theta_inv;
  std::vector<double> c1, c2;
};

Cheb coef(const Bounds& b, int degree) {
  Cheb k;
  const double theta = 0.5 * (b.hi + b.lo), delta = 0.5 * (b.hi - b.lo);
  k.theta_inv = 1.0 / theta;
  const double sigma1 = theta / delta;
  double rho = 1.0 / sigma1;
  for (int j = 1; j < degree; ++j) {
    const double rn = 1.0 / (2.0 * sigma1 - rho);
    k.c1.push_back(rn * rho);
    k.c2.push_back(2.0 * rn / delta);
    rho = rn;
  }
  return k;
}

template <class T>
T* wsp(stokes_ctx* c, const std::string& name, int64_t n) {
  return static_cast<T*>(c->workspace(name + (std::is_same<T, float>::value ? "_f" : "_d"), n * sizeof(T)));
}


// y[row][w] (+)= sum_k vals[k] x[cols[k]][w] over CSR rows (grid transfers
// of the velocity multigrid, W interleaved components per node)
template <typename T, int W, int ACC>
__global__ __launch_bounds__(kBlock) void k_csr_w(int64_t nrows, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ cols, const T* __restrict__ vals,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  GRID_STRIDE_ROWS(row, nrows) {
    T acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = ACC ? y[row * W + w] : T(0);
    for (int32_t k = rp[row]; k < rp[row + 1]; ++k) {
      const T v = vals[k];
      const T* xp = x + (int64_t)cols[k] * W;
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] = fma(v, xp[w], acc[w]);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) y[row * W + w] = acc[w];
  }
}

// y[i][w] = sum_j Cinv[i][j] x[j][w]: one wavefront per row
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_dense_mv_w(int64_t n, const T* __restrict__ Ci, const T* __restrict__ x,
                                                       T* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (row >= n) return;  // whole wavefronts exit together
  double acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0;
  for (int64_t j = lane; j < n; j += 64) {
    const double a = Ci[row * n + j];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] += a * (double)x[j * W + w];
  }
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = wave_sum(acc[w]);
  if (lane == 0)
#pragma unroll
    for (int w = 0; w < W; ++w) y[row * W + w] = (T)acc[w];
}

template <class F>
void dispatch_w_mg(int W, F&& f) {
  switch (W) {
    case 2: f(IC<2>{}); break;
    case 3: f(IC<3>{}); break;
    case 4: f(IC<4>{}); break;
    case 6: f(IC<6>{}); break;
    case 8: f(IC<8>{}); break;
    case 12: f(IC<12>{}); break;
    case 16: f(IC<16>{}); break;
    case 24: f(IC<24>{}); break;
    default: throw Error(STOKES_ERR_UNSUPPORTED, "velocity multigrid width");
  }
}

// dense symmetric matrix of a scalar sliced-ELL operator (host)
std::vector<double> sell_dense(stokes_ctx* c, const Sell& S, const DevBuf& v64) {
  const int64_t nr = S.nrows;
  std::vector<int64_t> sp(S.nslices + 1);
  std::vector<int32_t> cols(S.nnz_pad);
  std::vector<double> vals(S.nnz_pad);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HIP_CHECK(hipMemcpy(sp.data(), S.slice_ptr.p, sp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(cols.data(), S.cols.p, cols.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(vals.data(), v64.p, vals.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> A(nr * nr, 0.0);
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t k = sp[r / 64] + r % 64; k < sp[r / 64 + 1]; k += 64) A[r * nr + cols[k]] += vals[k];
  return A;
}
}  // namespace

// Dense inverse of the coarsest level when it is small enough.
static void dense_coarsest(stokes_ctx* c, MgHier& H) {
  const MgHier::View& V = H.lv.back();
  const Sell& S = *V.S;
  const int64_t nr = S.nrows;
  H.dense_n = 0;
  if (nr > c->mg_dense_max) return;
  std::vector<int64_t> sp(S.nslices + 1);
  std::vector<int32_t> cols(S.nnz_pad);
  std::vector<double> vals(S.nnz_pad);
  HIP_CHECK(hipStreamSynchronize(c->stream));
  HIP_CHECK(hipMemcpy(sp.data(), S.slice_ptr.p, sp.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(cols.data(), S.cols.p, cols.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  HIP_CHECK(hipMemcpy(vals.data(), V.v64->p, vals.size() * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<double> A(nr * nr, 0.0);
  for (int64_t r = 0; r < nr; ++r)
    for (int64_t k = sp[r / 64] + r % 64; k < sp[r / 64 + 1]; k += 64) A[r * nr + cols[k]] += vals[k];
  const std::vector<double> inv = spd_inverse(A, nr);
  std::vector<float> inv32(inv.begin(), inv.end());
  upload(H.cinv64, inv);
  upload(H.cinv32, inv32);
  H.dense_n = nr;
}

// Entry-split lanes per level (Sell::es).  The coarse levels have a few
// thousand rows of a two-ring stencil, where one lane per row leaves the chip
// idle.  mg_es = 1 (default): 8 lanes per row on levels below 2^14 rows, one
// lane above -- a fixed rule, so that every context sums the same way and
// solves are reproducible bit for bit; -1: time the level product in the form
// the FP32 V-cycle uses (half values when present) for E = 1, 2, 4, 8, 16
// and keep the fastest; 0: one lane per row; 2, 4, 8, 16: that E everywhere.
namespace {
void tune_levels(stokes_ctx* c, MgHier& H) {
  if (c->mg_es == 0) return;
  if (c->mg_es == 1) {
    for (auto& L : H.own) L->S.es = L->S.nrows < (int64_t(1) << 14) ? 8 : 1;
    return;
  }
  if (c->mg_es > 1) {  // a fixed E on every level
    for (auto& L : H.own) L->S.es = c->mg_es;
    return;
  }
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  for (auto& L : H.own) {
    Sell& S = L->S;
    if (S.nrows == 0) continue;
    DevBuf x, y;
    x.alloc(S.nrows * sizeof(float));
    y.alloc(S.nrows * sizeof(float));
    HIP_CHECK(hipMemsetAsync(x.p, 0, S.nrows * sizeof(float), c->stream));
    const bool half = c->pmg_half && L->v16.p;
    auto run = [&]() {
      if (half)
        ops::spmv_hs(c, S, L->v16.as<_Float16>(), L->s16, 1, x.as<float>(), y.as<float>(), 1.0f, nullptr, 0.0f);
      else
        ops::spmv<float>(c, S, L->v32.as<float>(), 1, x.as<float>(), y.as<float>(), 1.0f, nullptr, 0.0f);
    };
    int best = 1;
    float best_ms = 1e30f;
    for (int e : {1, 2, 4, 8, 16}) {
      S.es = e;
      run();  // warm-up
      HIP_CHECK(hipEventRecord(e0, c->stream));
      for (int rep = 0; rep < 5; ++rep) run();
      HIP_CHECK(hipEventRecord(e1, c->stream));
      HIP_CHECK(hipEventSynchronize(e1));
      float ms = 0;
      HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (const char* ev = std::getenv("STOKES_LOG"); ev && std::atoi(ev) >= 1)
        std::fprintf(stderr, "[stokes] mg level n=%d rows=%lld E=%d: %.1f us per product\n", L->n,
                     (long long)S.nrows, e, 1e3 * ms / 5);
      if (ms < best_ms) {
        best_ms = ms;
        best = e;
      }
    }
    S.es = best;
  }
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
}
}  // namespace

// Build both hierarchies (called once per context after assembly).  Level
// 0 is the pressure space: the (n+1)^dim vertices of the mesh for P2/P1, the
// (2n+1)^dim P2 nodes for P3/P2.  The P2 nodes of the mesh with n cells sit
// where the vertices of the mesh with 2n cells would, and a P1 function of
// the mesh is a P2 function with the nodal values that the Kuhn P1
// interpolation from n to 2n gives (vertex values kept, edge midpoints the
// mean of the two ends): so the P2 level is level "2n" of the same
// hierarchy, and its first coarse level is the P1 space of the mesh itself.
void build_mg(stokes_ctx* c) {
  MgHier& H = c->mgq;
  H.lv.clear();
  H.own.clear();
  const HostMesh& fm = c->mesh;
  const int D = fm.dim;
  int n = fm.order == 3 ? 2 * fm.n : fm.n;  // lattice intervals per side of the pressure nodes
  H.lv.push_back({&c->sQ, &c->XQ64, &c->XQ32, &c->dXQ64, &c->dXQ32, &c->bXQ_smooth, &c->bXQ, n});
  // coarsen while the current level is too large for the dense coarse solve
  while (n % 2 == 0 && n > 2 && ipow(n + 1, D) > c->mg_dense_max) {
    n /= 2;
    const int stride = fm.n / n;  // mesh vertices per coarse cell side
    auto L = std::make_unique<MgLevel>();
    L->n = n;
    HostMesh m;
    build_mesh(D, n, 0, 0.0, m);
    // coordinates: the level-0 vertex at stride * (grid index)
    const int64_t nf1 = fm.n + 1;
    for (int64_t g = 0; g < m.n_p1; ++g) {
      int64_t rem = g, fid = 0, st = 1;
      for (int d = 0; d < D; ++d, st *= nf1) {
        fid += (rem % (n + 1)) * stride * st;
        rem /= (n + 1);
      }
      for (int d = 0; d < D; ++d) m.vcoords[g * D + d] = fm.vcoords[fid * D + d];
    }
    L->nrows = m.n_p1;
    assemble_p1(c, m, *L);
    H.lv.push_back({&L->S, &L->v64, &L->v32, &L->d64, &L->d32, &L->bs, &L->bf, n});
    H.own.push_back(std::move(L));
  }
  dense_coarsest(c, H);
  // The Galerkin hierarchy of B_I Lambda_V^-1 B_I^T + M_Q.  On the P2
  // pressure of a P3/P2 pair that operator is close to the P2 mass matrix,
  // whose low-energy modes include non-smooth ones (vertex and edge values
  // coupled through negative entries) that the P1 coarse space does not
  // hold and that the smoothing interval leaves out, so its V-cycle
  // contracts more slowly there (about 0.72 per cycle on a 3D mesh), yet it
  // stays symmetric positive definite and is the better preconditioner.
  c->mgx.lv.clear();
  c->mgx.own.clear();
  c->mgx.dense_n = 0;
  if (fm.order != 3 || c->mgx_p3) {
    assemble_galerkin(c, c->mgx);
    dense_coarsest(c, c->mgx);
  }
  tune_levels(c, c->mgq);
  tune_levels(c, c->mgx);
}

template <class T>
void mg_vcycle(stokes_ctx* c, const MgHier& H, int nrb, const T* r, T* e, int lv) {
  const int nlev = static_cast<int>(H.lv.size());
  if (lv >= nlev) throw Error(STOKES_ERR_STATE, "pressure multigrid hierarchy not built");
  const MgHier::View& V = H.lv[lv];
  const Sell& S = *V.S;
  const T* vals = ops::pick<T>(*V.v64, *V.v32);
  const T* dinv = ops::pick<T>(*V.d64, *V.d32);
  const Bounds& bs = *V.bs;
  const Bounds& bf = *V.bf;
  const int64_t nr = S.nrows, n = nr * nrb;
  const std::string tag = "mg" + std::to_string(lv);
  T* d0 = wsp<T>(c, tag + "_d0", n);
  T* d1 = wsp<T>(c, tag + "_d1", n);
  T* res = wsp<T>(c, tag + "_res", n);
  // FP32 cycles read the half-precision level values (X = s16 x stored)
  const _Float16* v16 = nullptr;
  if constexpr (std::is_same<T, float>::value)
    if (c->pmg_half && V.v16 && V.v16->p) v16 = V.v16->as<_Float16>();
  // t = r - X e
  auto residual = [&](const T* e_, const T* r_, T* t_) {
    if constexpr (std::is_same<T, float>::value) {
      if (v16) return ops::spmv_hs(c, S, v16, V.s16, nrb, e_, t_, -1.0f, r_, 1.0f);
    }
    ops::spmv<T>(c, S, vals, nrb, e_, t_, (T)-1, r_, (T)1);
  };
  // z (+)= p(D^{-1} X) D^{-1} rin ; accumulate into z when acc != 0 (degree >= 2)
  auto cheb = [&](const Bounds& b, int degree, const T* rin, T* z, int acc) {
    const Cheb k = coef(b, degree);
    if (degree == 1) {
      ops::cheb_init<T>(c, nr, nrb, rin, dinv, (T)k.theta_inv, d0, z);
      return;
    }
    if constexpr (std::is_same<T, float>::value) {
      if (v16) {
        ops::cheb_first_hs(c, S, v16, V.s16, nrb, rin, dinv, (float)k.theta_inv, d0, res, z, (float)k.c1[0],
                           (float)k.c2[0], acc);
        float* da = d0;
        float* db = d1;
        for (int j = 2; j < degree; ++j) {
          ops::cheb_step_hs(c, S, v16, V.s16, nrb, da, db, res, res, z, dinv, (float)k.c1[j - 1], (float)k.c2[j - 1]);
          std::swap(da, db);
        }
        return;
      }
    }
    ops::cheb_first<T>(c, S, vals, nrb, rin, dinv, (T)k.theta_inv, d0, res, z, (T)k.c1[0], (T)k.c2[0], acc);
    T* da = d0;
    T* db = d1;
    for (int j = 2; j < degree; ++j) {
      ops::cheb_step<T>(c, S, vals, nrb, da, db, res, res, z, dinv, (T)k.c1[j - 1], (T)k.c2[j - 1], nullptr, nullptr,
                        1, 0, 0);
      std::swap(da, db);
    }
  };
  if (lv == nlev - 1) {  // coarsest: dense inverse, or a polynomial over the whole spectrum
    if (H.dense_n == nr) {
      const T* Ci = ops::pick<T>(H.cinv64, H.cinv32);
      dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
        constexpr int N = decltype(Nc)::value;
        (void)Dc;
        hipLaunchKernelGGL((k_dense_mv<T, N>), dim3((nr + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                           c->stream, nr, Ci, r, e);
      });
      ops::check_launch();
      ops::count_bytes(c, double(nr) * nr * sizeof(T) + 2.0 * nr * nrb * sizeof(T));  // dense inverse, r, e
    } else {
      cheb(bf, c->mg_coarse_degree, r, e, 0);
    }
    return;
  }
  const int nu = V.nu > 0 ? V.nu : c->mg_smooth_degree;
  T* t = wsp<T>(c, tag + "_t", n);
  const MgHier::View& C = H.lv[lv + 1];
  const int nf = V.n;
  const int64_t ncn = C.S->nrows * nrb;
  T* rc = wsp<T>(c, "mg" + std::to_string(lv + 1) + "_rc", ncn);
  T* ec = wsp<T>(c, "mg" + std::to_string(lv + 1) + "_ec", ncn);
  cheb(bs, nu, r, e, 0);                                                // pre-smoothing from zero
  residual(e, r, t);                                                    // t = r - X e
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int DD = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_restrict<T, DD, N>), dim3(ops::grid_for(C.S->nrows)), dim3(kBlock), 0, c->stream, nf, C.n,
                       (const T*)t, rc);
  });
  ops::check_launch();
  ops::count_bytes(c, double(n + ncn) * sizeof(T));  // fine residual read, coarse one written
  mg_vcycle<T>(c, H, nrb, rc, ec, lv + 1);
  dispatch_dn(c->dim, nrb, [&](auto Dc, auto Nc) {
    constexpr int DD = decltype(Dc)::value, N = decltype(Nc)::value;
    hipLaunchKernelGGL((k_prolong_add<T, DD, N>), dim3(ops::grid_for(nr)), dim3(kBlock), 0, c->stream, nf, C.n,
                       (const T*)ec, e);
  });
  ops::check_launch();
  ops::count_bytes(c, double(ncn + 2 * n) * sizeof(T));  // coarse correction read, e read and written
  residual(e, r, t);                                                    // t = r - X e
  if (nu >= 2) {
    cheb(bs, nu, t, e, 1);                                              // post-smoothing, e += p(.) t
  } else {
    T* dz = wsp<T>(c, tag + "_dz", n);
    cheb(bs, nu, t, dz, 0);
    ops::axpby<T>(c, n, (T)1, dz, (T)1, e);
  }
}

template void mg_vcycle<double>(stokes_ctx*, const MgHier&, int, const double*, double*, int);
template void mg_vcycle<float>(stokes_ctx*, const MgHier&, int, const float*, float*, int);

// ======================================================= velocity multigrid
//
// Geometric multigrid for the scalar velocity block alpha M + mu L (the
// A~_{lambda,3} preconditioner of Sec. 3.2) on the nested Kuhn meshes n, n/2,
// ...: the counterpart of the paper's fixed number of AMG V-cycles (Sec. 3.3).
//   * level 0 is the assembled interior operator (internal row order), the
//     coarse levels rediscretise alpha M + mu L on the coarse meshes (their
//     vertices keep the fine jittered positions);
//   * interpolation is P2 interpolation of the coarse basis at the fine P2
//     nodes (exact for the nested unjittered meshes), restriction its
//     transpose, coarse Dirichlet nodes dropped;
//   * Chebyshev-Jacobi smoothing on the upper spectrum, the same polynomial
//     before and after the correction, so the cycle is symmetric positive
//     definite; the coarsest level (<= mg_dense_max rows) is solved densely.

void build_vmg(stokes_ctx* c) {
  c->vmg.clear();
  c->vmg_dense_n = 0;
  const HostMesh& fm = c->mesh;
  const int D = fm.dim;
  int nf = fm.n, stride = 1;
  std::vector<int32_t> fine_nat = c->h_int2nat;
  auto rows_of = [&](int n) { return ipow(2 * int64_t(n) - 1, D); };
  while (nf % 2 == 0 && nf >= 4 && rows_of(nf) > c->mg_dense_max) {
    const int nc = nf / 2;
    stride *= 2;
    auto L = std::make_unique<VmgLevel>();
    L->n = nc;
    HostMesh m;
    build_mesh(D, nc, 0, 0.0, m);
    const int64_t nf1 = fm.n + 1;
    for (int64_t g = 0; g < m.n_p1; ++g) {
      int64_t rem = g, fid = 0, st = 1;
      for (int d = 0; d < D; ++d, st *= nf1) {
        fid += (rem % (nc + 1)) * stride * st;
        rem /= (nc + 1);
      }
      for (int d = 0; d < D; ++d) m.vcoords[g * D + d] = fm.vcoords[fid * D + d];
    }
    assemble_p2_level(c, m, *L);
    HostCsr P, R;
    std::vector<double> pv;
    p2_prolongation(D, nf, fine_nat, P, pv);
    std::vector<int64_t> tsrc;
    transpose_pattern(P, R, tsrc);
    std::vector<double> rv(tsrc.size());
    for (size_t k = 0; k < tsrc.size(); ++k) rv[k] = pv[tsrc[k]];
    auto up = [&](const HostCsr& h, const std::vector<double>& v, DevCsr& d, DevBuf& v64, DevBuf& v32) {
      std::vector<int32_t> rp(h.rowptr.begin(), h.rowptr.end());
      d.nrows = h.nrows;
      d.nnz = h.rowptr.back();
      upload(d.rowptr, rp);
      upload(d.cols, h.cols);
      upload(v64, v);
      std::vector<float> f(v.begin(), v.end());
      upload(v32, f);
    };
    up(P, pv, L->P, L->pv64, L->pv32);
    up(R, rv, L->R, L->rv64, L->rv32);
    // natural ids of the coarse interior nodes, the rows of the next level
    fine_nat.clear();
    for (int64_t v = 0; v < m.n_p2; ++v)
      if (!m.p2_bnd[v]) fine_nat.push_back(static_cast<int32_t>(v));
    c->vmg.push_back(std::move(L));
    nf = nc;
  }
  // coarsest level: dense inverse when small
  if (!c->vmg.empty()) {
    VmgLevel& L = *c->vmg.back();
    if (L.nrows <= c->mg_dense_max) {
      const std::vector<double> inv = spd_inverse(sell_dense(c, L.S, L.v64), L.nrows);
      std::vector<float> inv32(inv.begin(), inv.end());
      upload(c->vmg_cinv64, inv);
      upload(c->vmg_cinv32, inv32);
      c->vmg_dense_n = L.nrows;
    }
  } else if (c->n_int <= c->mg_dense_max) {
    const std::vector<double> inv = spd_inverse(sell_dense(c, c->sA, c->A64), c->n_int);
    std::vector<float> inv32(inv.begin(), inv.end());
    upload(c->vmg_cinv64, inv);
    upload(c->vmg_cinv32, inv32);
    c->vmg_dense_n = c->n_int;
  }
  HIP_CHECK(hipStreamSynchronize(c->stream));
  c->vmg_mu = c->prob.mu;
  c->vmg_built = true;
}

template <class T>
void vel_vcycle(stokes_ctx* c, int W, const T* r, T* e, int lv) {
  const int nlev = static_cast<int>(c->vmg.size()) + 1;
  const bool fine = lv == 0;
  const VmgLevel* L = fine ? nullptr : c->vmg[lv - 1].get();
  const Sell& S = fine ? c->sA : L->S;
  const T* vals = fine ? ops::pick<T>(c->A64, c->A32) : ops::pick<T>(L->v64, L->v32);
  const T* dinv = fine ? ops::pick<T>(c->dA64, c->dA32) : ops::pick<T>(L->d64, L->d32);
  const Bounds bf = fine ? c->bA : L->bf;
  const Bounds bs = fine ? Bounds{c->bA.hi / c->mg_smooth_ratio, c->bA.hi} : L->bs;
  const int64_t nr = S.nrows, n = nr * W;
  const std::string tag = "vmg" + std::to_string(lv);
  T* d0 = wsp<T>(c, tag + "_d0", n);
  T* d1 = wsp<T>(c, tag + "_d1", n);
  T* res = wsp<T>(c, tag + "_res", n);
  auto cheb = [&](const Bounds& b, int degree, const T* rin, T* z, int acc) {
    const Cheb k = coef(b, degree);
    ops::cheb_first<T>(c, S, vals, W, rin, dinv, (T)k.theta_inv, d0, res, z, (T)k.c1[0], (T)k.c2[0], acc);
    T* da = d0;
    T* db = d1;
    for (int j = 2; j < degree; ++j) {
      ops::cheb_step<T>(c, S, vals, W, da, db, res, res, z, dinv, (T)k.c1[j - 1], (T)k.c2[j - 1], nullptr, nullptr, 1,
                        0, 0);
      std::swap(da, db);
    }
  };
  if (lv == nlev - 1) {  // coarsest
    if (c->vmg_dense_n == nr) {
      const T* Ci = ops::pick<T>(c->vmg_cinv64, c->vmg_cinv32);
      dispatch_w_mg(W, [&](auto Wc) {
        constexpr int WW = decltype(Wc)::value;
        hipLaunchKernelGGL((k_dense_mv_w<T, WW>), dim3((nr + kBlock / 64 - 1) / (kBlock / 64)), dim3(kBlock), 0,
                           c->stream, nr, Ci, r, e);
      });
      ops::check_launch();
      ops::count_bytes(c, double(nr) * nr * sizeof(T) + 2.0 * nr * W * sizeof(T));
    } else {
      cheb(bf, c->mg_coarse_degree, r, e, 0);
    }
    return;
  }
  const VmgLevel& C = *c->vmg[lv];
  const int nu = std::max(2, c->vmg_smooth_degree);
  T* t = wsp<T>(c, tag + "_t", n);
  const int64_t ncn = C.nrows * W;
  T* rc = wsp<T>(c, "vmg" + std::to_string(lv + 1) + "_rc", ncn);
  T* ec = wsp<T>(c, "vmg" + std::to_string(lv + 1) + "_ec", ncn);
  cheb(bs, nu, r, e, 0);                                 // pre-smoothing from zero
  ops::spmv<T>(c, S, vals, W, e, t, (T)-1, r, (T)1);     // t = r - A e
  dispatch_w_mg(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    hipLaunchKernelGGL((k_csr_w<T, WW, 0>), dim3(ops::grid_for(C.nrows)), dim3(kBlock), 0, c->stream, C.nrows,
                       C.R.rowptr.as<int32_t>(), C.R.cols.as<int32_t>(), ops::pick<T>(C.rv64, C.rv32), (const T*)t, rc);
  });
  ops::check_launch();
  // CSR restriction: row pointers, columns and values, fine residual gathered, coarse written
  ops::count_bytes(c, double(C.nrows + 1) * 4.0 + double(C.R.nnz) * (4.0 + sizeof(T)) + double(n + ncn) * sizeof(T));
  vel_vcycle<T>(c, W, rc, ec, lv + 1);
  dispatch_w_mg(W, [&](auto Wc) {
    constexpr int WW = decltype(Wc)::value;
    hipLaunchKernelGGL((k_csr_w<T, WW, 1>), dim3(ops::grid_for(nr)), dim3(kBlock), 0, c->stream, nr,
                       C.P.rowptr.as<int32_t>(), C.P.cols.as<int32_t>(), ops::pick<T>(C.pv64, C.pv32), (const T*)ec, e);
  });
  ops::check_launch();
  ops::count_bytes(c, double(nr + 1) * 4.0 + double(C.P.nnz) * (4.0 + sizeof(T)) + double(ncn + 2 * n) * sizeof(T));
  ops::spmv<T>(c, S, vals, W, e, t, (T)-1, r, (T)1);     // t = r - A e
  cheb(bs, nu, t, e, 1);                                 // post-smoothing, e += p(.) t
}

template void vel_vcycle<double>(stokes_ctx*, int, const double*, double*, int);
template void vel_vcycle<float>(stokes_ctx*, int, const float*, float*, int);

}  // namespace stokes

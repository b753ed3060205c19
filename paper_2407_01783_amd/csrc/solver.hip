// Krylov solvers of the generalized Stokes system.
//
//   * inner velocity solve A~^{-1}: PCG (one system per component and
//     right-hand side; one joint system per right-hand side when the
//     augmented-Lagrangian term couples the components) preconditioned by a
//     Chebyshev-Jacobi polynomial of A = alpha M + mu L (the paper's
//     A~_{lambda,3}, Sec. 3.2), or the polynomial alone (fixed mode);
//   * Cahouet-Chabard preconditioner of the Schur complement (Sec. 4.1):
//     C = alpha X^{-1} + mu (1 + gamma) M_Q^{-1}, X in {L_Q, B Lambda^{-1} B^T,
//     B M^{-1} B^T}, X^{-1} by PCG preconditioned with Chebyshev-Jacobi on
//     eps M_Q + L_Q (eps = 1, Sec. 4.2);
//   * Method 1 (Sec. 2.3): flexible CG on S = B A^{-1} B^T;
//   * Method 2 (Sec. 2.4): right-preconditioned flexible GMRES(m) on the
//     coupled matrix with the block preconditioners of Sec. 2.4 / 6.2,
//     classical Gram-Schmidt with re-orthogonalisation (CGS2);
//   * an FP64 refinement loop around either: true residual of the coupled
//     system, correction solve (inner precision FP32 in mixed mode), update.
//
// All vectors are in the internal layout (see kernels.h); scalars of the
// inner CG live on the device, outer Krylov scalars on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <type_traits>

#include "kernels.h"
#include "ops.h"
#include "solver.h"

namespace stokes {

namespace {

// FGMRES: the next step's preconditioner is queued ahead of the host's
// rotations while the residual estimate is above this multiple of the goal
// (a step shrinks it by about 5x on the benchmark problems, so the step in
// flight is then almost surely not the last).
constexpr double kQueueAhead = 30.0;

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

struct ChebCoef {
  double theta_inv = 1;
  std::vector<double> c1, c2;  // steps 1..k-1
};

// Coefficients of the Chebyshev iteration on [lo, hi] (Saad, Iterative
// Methods for Sparse Linear Systems, Alg. 12.1).
ChebCoef cheb_coef(const Bounds& b, int degree) {
  ChebCoef k;
  const double theta = 0.5 * (b.hi + b.lo), delta = 0.5 * (b.hi - b.lo);
  k.theta_inv = 1.0 / theta;
  if (degree <= 1) return k;
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

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// STOKES_LOG=1: one line per refinement sweep / Krylov cycle on stderr;
// STOKES_LOG=2 adds every inner solve.
int log_level() {
  static int lv = [] {
    const char* e = std::getenv("STOKES_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return lv;
}

}  // namespace

// ======================================================================
template <class T>
class Engine {
 public:
  Engine(stokes_ctx* c, const stokes_solve_opts& o, int nrb, SolveStats& st)
      : c_(c), o_(o), nrb_(nrb), D_(c->dim), W_(c->dim * nrb), st_(st) {
    gamma_ = c->prob.gamma;
    mu_ = c->prob.mu;
    alpha_ = c->prob.alpha;
    const bool f32 = std::is_same<T, float>::value;
    al_deg_ = f32 ? 18 : 26;  // M_Q^{-1} inside A_gamma: 2 * 0.382^k below 1e-7 / 1e-11
    // mu (1 + gamma) M_Q^{-1} term of the Cahouet-Chabard operator: next to
    // alpha X^{-1} it weighs at most about mu (1 + gamma) / (alpha h^2) on the
    // finest pressure modes, so a low-degree polynomial suffices when that
    // ratio is small (unsteady, small-viscosity regime)
    const double h = 1.0 / std::max(1, c->mesh.n);
    cc_mq_deg_ = mu_ * (1.0 + gamma_) / (alpha_ * h * h) < 0.1 ? 2 : 6;
    mv_deg_ = 8;              // M_V^{-1} inside B M^{-1} B^T
  }

  // ------------------------------------------------------------ buffers
  T* buf(const std::string& name, int64_t n) {
    return static_cast<T*>(c_->workspace(name + (std::is_same<T, float>::value ? "_f" : "_d"), n * sizeof(T)));
  }
  int64_t nu() const { return c_->n_int * W_; }
  int64_t np() const { return c_->n_p1 * nrb_; }

  const T* A() const { return ops::pick<T>(c_->A64, c_->A32); }
  void no_augmented_lagrangian() { gamma_ = 0; }
  const T* dA() const { return ops::pick<T>(c_->dA64, c_->dA32); }
  Scalars* scal(int i) { return c_->scal.as<Scalars>() + i; }

  // ------------------------------------------------------- Chebyshev
  // z = p_k(D^{-1} S) D^{-1} r  (k = degree), buffers tagged by `tag`
  void cheb_apply(const std::string& tag, const Sell& S, const T* vals, const T* dinv, const Bounds& b, int degree,
                  int W, const T* r, T* z) {
    const int64_t n = S.nrows * W;
    const ChebCoef k = cheb_coef(b, degree);
    T* d0 = buf(tag + "_d0", n);
    T* d1 = buf(tag + "_d1", n);
    T* res = buf(tag + "_res", n);
    if (degree <= 1) {
      ops::cheb_init<T>(c_, S.nrows, W, r, dinv, (T)k.theta_inv, d0, z);
      return;
    }
    if constexpr (std::is_same<T, float>::value) {
      // FP32 velocity block: read the half-precision copy of A_II D^{-1}
      if (&S == &c_->sA && vals == A() && c_->vel_half && c_->AD16.p && c_->vel_bf) {
        // the direction in bfloat16 (the float buffers hold it, narrower)
        uint16_t* q0 = reinterpret_cast<uint16_t*>(d0);
        uint16_t* q1 = reinterpret_cast<uint16_t*>(d1);
        if (c_->cheb_defer && degree >= 3 && degree - 2 <= kQSumMax) {
          // z = D^{-1} (theta_inv r + q_1 + ... + q_{degree-1}) formed by the
          // last step: the steps before it neither read nor write z, and
          // each keeps its direction q_j (buffers q_1 .. q_{degree-2})
          std::vector<uint16_t*> q(degree - 1, nullptr);
          for (int j = 1; j <= degree - 2; ++j)
            q[j] = reinterpret_cast<uint16_t*>(buf(tag + "_q" + std::to_string(j), n));
          ops::cheb_first_hb(c_, W, r, dinv, (float)k.theta_inv, q[1], res, z, (float)k.c1[0], (float)k.c2[0],
                             false);
          for (int j = 2; j < degree - 1; ++j)
            ops::cheb_step_hb(c_, W, q[j - 1], q[j], res, res, z, dinv, (float)k.c1[j - 1], (float)k.c2[j - 1],
                              nullptr, false);
          QSum fin{};
          fin.r = reinterpret_cast<const float*>(r);
          fin.theta_inv = (float)k.theta_inv;
          fin.n = degree - 2;
          for (int j = 1; j <= degree - 2; ++j) fin.q[j - 1] = q[j];
          ops::cheb_step_hb(c_, W, q[degree - 2], nullptr, res, nullptr, z, dinv, (float)k.c1[degree - 2],
                            (float)k.c2[degree - 2], &fin);
          return;
        }
        ops::cheb_first_hb(c_, W, r, dinv, (float)k.theta_inv, q0, res, z, (float)k.c1[0], (float)k.c2[0]);
        for (int j = 2; j < degree; ++j) {
          ops::cheb_step_hb(c_, W, q0, q1, res, res, z, dinv, (float)k.c1[j - 1], (float)k.c2[j - 1]);
          std::swap(q0, q1);
        }
        return;
      }
      if (&S == &c_->sA && vals == A() && c_->vel_half && c_->AD16.p) {
        ops::cheb_first_h(c_, W, r, dinv, (float)k.theta_inv, d0, res, z, (float)k.c1[0], (float)k.c2[0]);
        for (int j = 2; j < degree; ++j) {
          ops::cheb_step_h(c_, W, d0, d1, res, res, z, dinv, (float)k.c1[j - 1], (float)k.c2[j - 1]);
          std::swap(d0, d1);
        }
        return;
      }
    }
    ops::cheb_first<T>(c_, S, vals, W, r, dinv, (T)k.theta_inv, d0, res, z, (T)k.c1[0], (T)k.c2[0]);
    for (int j = 2; j < degree; ++j) {
      ops::cheb_step<T>(c_, S, vals, W, d0, d1, res, res, z, dinv, (T)k.c1[j - 1], (T)k.c2[j - 1], nullptr, nullptr,
                        1, 0, 0);
      std::swap(d0, d1);
    }
  }

  // ------------------------------------------------------------ PCG
  struct Op {
    const Sell* S = nullptr;  // fused scalar SELL operator, or
    std::function<void(const T*, T*)> apply;  // composite t = X z
    std::function<void(const T*, T*)> extra;  // added term (augmented Lagrangian)
  };
  struct Prec {
    const Sell* S;
    const T* vals;
    const T* dinv;
    Bounds b;
    int degree;
    std::function<void(const T*, T*)> apply;  // general preconditioner z = M^{-1} r
  };

  // Solve op x = b per system to ||r|| <= rtol ||b||; returns iterations.
  // graph = true replays the iteration body as a captured graph (worth it for
  // the many short kernels of the pressure solve).
  // fixed > 0 runs exactly that many iterations without convergence checks.
  int pcg(const std::string& tag, const Op& op, const T* opvals, const Prec& pc, int64_t nrows, int W, int cps,
          const T* b, T* x, double rtol, int maxit, int sc_index, bool graph, int fixed = 0) {
    const int64_t n = nrows * W;
    const int nsys = W / cps;
    Scalars* sc = scal(sc_index);
    T* r = buf(tag + "_r", n);
    T* z = buf(tag + "_z", n);
    T* p = buf(tag + "_p", n);
    T* q = buf(tag + "_q", n);
    T* d0 = buf(tag + "_d0", n);
    T* d1 = buf(tag + "_d1", n);
    T* res = buf(tag + "_res", n);
    T* t = (op.apply || op.extra) ? buf(tag + "_t", n) : nullptr;
    ops::zero_dev(c_, x, n * sizeof(T));
    ops::zero_dev(c_, p, n * sizeof(T));
    ops::zero_dev(c_, q, n * sizeof(T));
    ops::copy_dev(c_, r, b, n * sizeof(T));
    double* slots = c_->red.result.as<double>() + 2 * kMaxSys;
    ops::dot_dev<T>(c_, nrows, W, b, nullptr, nullptr, slots);
    hipLaunchKernelGGL(k_scal_init, dim3(1), dim3(64), 0, c_->stream, sc, (const double*)slots, cps, nsys,
                       rtol * rtol);
    ops::check_launch();
    const ChebCoef k = cheb_coef(pc.b, pc.degree);
    const T thinv = pc.degree > 1 ? (T)k.theta_inv : (T)1;
    // z = M^{-1} r with rho = r . z
    auto precond = [&](bool first) {
      if (pc.apply) {
        pc.apply(r, z);
        ops::dot_dev<T>(c_, nrows, W, r, z, nullptr, slots);
        hipLaunchKernelGGL(k_scal_rho, dim3(1), dim3(64), 0, c_->stream, sc, (const double*)slots, cps, nsys,
                           first ? 1 : 0);
        ops::check_launch();
        return;
      }
      if (pc.degree <= 1) {
        ops::cheb_init<T>(c_, nrows, W, r, pc.dinv, thinv, d0, z);
        ops::dot_dev<T>(c_, nrows, W, r, z, nullptr, slots);
        hipLaunchKernelGGL(k_scal_rho, dim3(1), dim3(64), 0, c_->stream, sc, (const double*)slots, cps, nsys,
                           first ? 1 : 0);
        ops::check_launch();
        return;
      }
      if (first) ops::cheb_init<T>(c_, nrows, W, r, pc.dinv, thinv, d0, z);
      T* da = d0;
      T* db = d1;
      for (int j = 1; j < pc.degree; ++j) {
        const bool last = j == pc.degree - 1;
        ops::cheb_step<T>(c_, *pc.S, pc.vals, W, da, db, j == 1 ? r : res, res, z, pc.dinv, (T)k.c1[j - 1],
                          (T)k.c2[j - 1], last ? r : nullptr, sc, cps, nsys, first ? 1 : 0);
        std::swap(da, db);
      }
    };
    precond(true);
    // one CG iteration; converged systems are frozen on the device (alpha =
    // beta = 0), so several iterations can run between host checks, and the
    // fixed kernel sequence is replayed as a captured graph
    auto body = [&]() {
      if (op.apply) {
        op.apply(z, t);
        ops::cg_spmv<T>(c_, nrows, nullptr, nullptr, W, z, t, q, p, sc, cps, nsys);
      } else {
        if (op.extra) op.extra(z, t);
        ops::cg_spmv<T>(c_, nrows, op.S, opvals, W, z, op.extra ? t : nullptr, q, p, sc, cps, nsys);
      }
      if (pc.apply) {
        ops::cg_update<T>(c_, nrows, W, 2, x, r, p, q, pc.dinv, (T)1, d0, z, sc, cps, nsys);
        precond(false);
      } else if (pc.degree <= 1) {
        ops::cg_update<T>(c_, nrows, W, 1, x, r, p, q, pc.dinv, (T)1, d0, z, sc, cps, nsys);
      } else {
        ops::cg_update<T>(c_, nrows, W, 0, x, r, p, q, pc.dinv, thinv, d0, z, sc, cps, nsys);
        precond(false);
      }
    };
    char key[256];
    std::snprintf(key, sizeof(key), "pcg:%s:%d:%d:%p:%d:%d:%d", tag.c_str(), W, (int)sizeof(T), (void*)x, o_.schur_pc,
                  pc.degree, pc.apply ? 1 : 0);
    const int every = std::max(1, c_->cg_check_every);
    int it = 0;
    if (fixed > 0) {
      for (int i = 0; i < fixed; ++i) {
        if (graph) c_->run_graph(key, body);
        else body();
      }
      it = fixed;
      maxit = fixed;  // the check below only looks for breakdown
    }
    for (;;) {
      sync_scalars(sc_index);
      const Scalars& h = *c_->h_scal;
      if (h.breakdown) {
        std::string msg = "inner CG '" + tag + "' breakdown (non-positive curvature) at iteration " +
                          std::to_string(it) + ":";
        for (int s2 = 0; s2 < nsys; ++s2) {
          char b[160];
          std::snprintf(b, sizeof(b), " [sys %d rho %.3e sigma %.3e rr %.3e bb %.3e active %d]", s2, h.rho[s2],
                        h.sigma[s2], h.rr[s2], h.bb[s2], h.active[s2]);
          msg += b;
        }
        throw Error(STOKES_ERR_BREAKDOWN, msg);
      }
      bool any = false;
      for (int s = 0; s < nsys; ++s) any = any || h.active[s];
      if (!any || it >= maxit) {
        if (log_level() >= 2) {
          double worst = 0;
          for (int s2 = 0; s2 < nsys; ++s2)
            if (h.bb[s2] > 0) worst = std::max(worst, std::sqrt(h.rr[s2] / h.bb[s2]));
          std::fprintf(stderr, "[stokes]   pcg %s: %d its, max rel res %.3e\n", tag.c_str(), it, worst);
        }
        break;
      }
      const int k = std::min(every, maxit - it);
      for (int i = 0; i < k; ++i) {
        if (graph) c_->run_graph(key, body);
        else body();
      }
      it += k;
    }
    return it;
  }

  void sync_scalars(int i) {
    HIP_CHECK(hipMemcpyAsync(c_->h_scal, scal(i), sizeof(Scalars), hipMemcpyDeviceToHost, c_->stream));
    HIP_CHECK(hipStreamSynchronize(c_->stream));
  }

  // ------------------------------------------------- operator pieces
  // t = gamma mu B^T M_Q^{-1} B z   (augmented-Lagrangian term, Eq. "def_of_Alambda")
  void al_term(const T* z, T* t) {
    T* bp = buf("al_bz", np());
    T* y = buf("al_y", np());
    ops::Bmul<T>(c_, nrb_, z, bp, (T)1, nullptr, (T)0);
    cheb_apply("alq", c_->sQ, ops::pick<T>(c_->MQ64, c_->MQ32), ops::pick<T>(c_->dMQ64, c_->dMQ32), c_->bMQ, al_deg_,
               nrb_, bp, y);
    ops::Btmul<T>(c_, nrb_, y, nullptr, t, (T)(gamma_ * mu_), nullptr, (T)0);
  }

  // x = A~^{-1} b (velocity block)
  void vel_solve(const T* b, T* x) {
    ops::PhaseScope phase(c_, PHASE_VEL);
    Prec pc{&c_->sA, A(), dA(), c_->bA, std::max(1, o_.cheb_degree), {}};
    const bool mg = o_.vel_pc == STOKES_VEL_MG;
    if (mg) pc.apply = [this](const T* r, T* z) { vel_vcycle<T>(c_, W_, r, z, 0); };
    if (o_.inner_mode == STOKES_INNER_FIXED) {
      if (mg) vel_vcycle<T>(c_, W_, b, x, 0);
      else cheb_apply("vfx", c_->sA, A(), dA(), c_->bA, std::max(1, o_.cheb_degree), W_, b, x);
      return;
    }
    Op op;
    int cps = 1;
    if (c_->strain) {
      // alpha M + mu (L + D) couples the components; A~_{lambda,3} (the
      // vector-Laplacian block) stays the preconditioner, as in Sec. 3.2
      cps = D_;
      op.apply = [this](const T* z, T* t) {
        ops::velop<T>(c_, nrb_, z, t, (T)1, nullptr, (T)0);
        if (gamma_ > 0) {
          T* ta = buf("vs_al", nu());
          al_term(z, ta);
          ops::axpby<T>(c_, nu(), (T)1, ta, (T)1, t);
        }
      };
    } else {
      op.S = &c_->sA;
      if (gamma_ > 0) {
        op.extra = [this](const T* z, T* t) { al_term(z, t); };
        cps = D_;
      }
    }
    st_.inner_u += pcg("vcg", op, A(), pc, c_->n_int, W_, cps, b, x, o_.inner_rtol_u, o_.max_inner, 0, false,
                       o_.inner_its_u);
  }

  // x = M_Q^{-1} b by CG preconditioned with Chebyshev-Jacobi on the exact
  // element bounds of the Jacobi-scaled P1 mass (tolerance inner_rtol_p)
  void mq_solve(const T* b, T* x) {
    Op op;
    op.S = &c_->sQ;
    const Prec pc{&c_->sQ, ops::pick<T>(c_->MQ64, c_->MQ32), ops::pick<T>(c_->dMQ64, c_->dMQ32), c_->bMQ, 4, {}};
    st_.inner_p += pcg("pmq", op, ops::pick<T>(c_->MQ64, c_->MQ32), pc, c_->n_p1, nrb_, 1, b, x, o_.inner_rtol_p,
                       o_.max_inner, 1, true);
  }

  // t = X z for the Cahouet-Chabard family
  void x_apply(const T* z, T* t) {
    if (o_.schur_pc == STOKES_CC_LUMPED) {
      ops::spmv<T>(c_, c_->sX, ops::pick<T>(c_->XL64, c_->XL32), nrb_, z, t, (T)1, nullptr, (T)0);
    } else if (o_.schur_pc == STOKES_CC_MASS) {
      T* tu = buf("x_tu", nu());
      T* yu = buf("x_yu", nu());
      ops::Btmul<T>(c_, nrb_, z, nullptr, tu, (T)1, nullptr, (T)0);
      cheb_apply("mvc", c_->sA, ops::pick<T>(c_->MV64, c_->MV32), ops::pick<T>(c_->dMV64, c_->dMV32), c_->bMV,
                 mv_deg_, W_, tu, yu);
      ops::Bmul<T>(c_, nrb_, yu, t, (T)1, nullptr, (T)0);
    } else {
      ops::spmv<T>(c_, c_->sQ, ops::pick<T>(c_->LQ64, c_->LQ32), nrb_, z, t, (T)1, nullptr, (T)0);
    }
  }

  // x = X^{-1} b on the mean-free pressures; the preconditioner (fixed
  // mode: the approximation itself) is one pressure multigrid V-cycle
  void x_solve(const T* b, T* x) {
    Prec pc{&c_->sQ, ops::pick<T>(c_->XQ64, c_->XQ32), ops::pick<T>(c_->dXQ64, c_->dXQ32), c_->bXQ, 1, {}};
    // the Galerkin hierarchy for the lumped variant (when built), else the
    // V-cycle of eps M_Q + L_Q
    const MgHier& H =
        (o_.schur_pc == STOKES_CC_LUMPED && c_->use_mgx && !c_->mgx.lv.empty()) ? c_->mgx : c_->mgq;
    pc.apply = [this, &H](const T* r, T* z) { mg_vcycle<T>(c_, H, nrb_, r, z, 0); };
    if (o_.inner_mode == STOKES_INNER_FIXED) {
      mg_vcycle<T>(c_, H, nrb_, b, x, 0);
      return;
    }
    Op op;
    const T* opvals = nullptr;
    if (o_.schur_pc == STOKES_CC_LAPLACE) {
      op.S = &c_->sQ;
      opvals = ops::pick<T>(c_->LQ64, c_->LQ32);
    } else if (o_.schur_pc == STOKES_CC_LUMPED) {
      op.S = &c_->sX;  // B_I Lambda_V^-1 B_I^T assembled at setup
      opvals = ops::pick<T>(c_->XL64, c_->XL32);
    } else {
      op.apply = [this](const T* z, T* t) { x_apply(z, t); };
    }
    st_.inner_p += pcg("pcg", op, opvals, pc, c_->n_p1, nrb_, 1, b, x, o_.inner_rtol_p, o_.max_inner, 1, true,
                       o_.inner_its_p);
  }

  // z = C r = alpha X^{-1} r + mu (1 + gamma) M_Q^{-1} r on the mean-free
  // pressures (X is singular on constants: its inverse acts on 1-perp).
  // Inside the coupled preconditioner with fixed inner operators both
  // projections are skipped (mean_free = false): X^{-1} is then one V-cycle
  // (or polynomial) of the nonsingular eps M_Q + L_Q, the input already sums
  // to zero up to rounding (B u does for interior u, and the right-hand
  // side's pressure part is made mean-free), and a constant added to z_p
  // changes neither B^T z_p nor K z, only the pressure level that the final
  // normalization fixes.  Inner CGs on the singular X keep them.
  void cc_apply(const T* r, T* z, bool mean_free = true) {
    ops::PhaseScope phase(c_, PHASE_PRES);
    mean_free = mean_free || o_.inner_mode != STOKES_INNER_FIXED;
    T* y = buf("cc_y", np());
    const T* rin = r;
    if (mean_free) {
      T* rm = buf("cc_r", np());
      ops::remove_mean_into<T>(c_, nrb_, r, rm);
      rin = rm;
    }
    x_solve(rin, z);
    cheb_apply("ccq", c_->sQ, ops::pick<T>(c_->MQ64, c_->MQ32), ops::pick<T>(c_->dMQ64, c_->dMQ32), c_->bMQ,
               cc_mq_deg_, nrb_, rin, y);
    ops::axpby<T>(c_, np(), (T)(mu_ * (1.0 + gamma_)), y, (T)alpha_, z);
    if (mean_free) ops::remove_mean<T>(c_, nrb_, z);
  }

  // z = P^{-1} v, block preconditioners of the coupled matrix (Sec. 2.4);
  // bt (optional, upper triangular only) receives B^T z_p
  void block_prec(const T* vu, const T* vp, T* zu, T* zp, T* bt = nullptr) {
    T* tp = buf("bp_tp", np());
    T* tu = buf("bp_tu", nu());
    T* yu = buf("bp_yu", nu());
    if (o_.coupled_pc == STOKES_PC_UPPER) {
      cc_apply(vp, zp, false);
      ops::Btmul<T>(c_, nrb_, zp, nullptr, tu, (T)1, vu, (T)1, bt);  // tu = v_u + B^T z_p
      vel_solve(tu, zu);
      return;
    }
    vel_solve(vu, zu);                                            // y_u = A~^{-1} v_u
    ops::Bmul<T>(c_, nrb_, zu, tp, (T)-1, vp, (T)1);             // t_p = v_p - B y_u
    cc_apply(tp, zp, false);                                      // z_p = S~^{-1} t_p
    if (o_.coupled_pc == STOKES_PC_LOWER) return;
    ops::Btmul<T>(c_, nrb_, zp, nullptr, tu, (T)1, nullptr, (T)0);  // B^T z_p
    vel_solve(tu, yu);                                               // A~^{-1} B^T z_p
    ops::axpby<T>(c_, nu(), (T)1, yu, (T)1, zu);                      // z_u = y_u + ...
  }

  // ------------------------------------------------------- helpers
  // residual history: the largest per-right-hand-side estimate over ||b||
  void record_hist(const std::vector<double>& est) {
    double v = 0;
    for (size_t r = 0; r < est.size(); ++r) v = std::max(v, est[r] * (r < st_.inv_bn.size() ? st_.inv_bn[r] : 0.0));
    st_.hist.push_back(v);
  }

  template <class TX, class TY>
  void axpy_rhs(int64_t nrows, bool vel, const double* a, const double* b, const TX* x, TY* y) {
    Coef8 ca{}, cb{};
    for (int r = 0; r < 8; ++r) {
      ca.v[r] = r < nrb_ ? a[r] : 0;
      cb.v[r] = r < nrb_ ? b[r] : 0;
    }
    dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
      constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
      if (vel)
        hipLaunchKernelGGL((k_axpy_rhs<TX, TY, D * N, D>), dim3(ops::grid_for(nrows)), dim3(kBlock), 0, c_->stream,
                           nrows, ca, cb, x, y);
      else
        hipLaunchKernelGGL((k_axpy_rhs<TX, TY, N, 1>), dim3(ops::grid_for(nrows)), dim3(kBlock), 0, c_->stream,
                           nrows, ca, cb, x, y);
    });
    ops::check_launch();
    ops::count_bytes(c_, double(nrows) * (vel ? D_ * nrb_ : nrb_) * (sizeof(TX) + 2 * sizeof(TY)));
  }

  // per right-hand-side dots over (velocity, pressure) FP64 pieces
  std::vector<double> dots(const double* xu, const double* yu, const double* xp, const double* yp) {
    std::vector<double> out(nrb_, 0.0);
    if (xu) {
      auto s = ops::dot_host<double>(c_, c_->n_int, W_, xu, yu);
      for (int w = 0; w < W_; ++w) out[w / D_] += s[w];
    }
    if (xp) {
      auto s = ops::dot_host<double>(c_, c_->n_p1, nrb_, xp, yp);
      for (int r = 0; r < nrb_; ++r) out[r] += s[r];
    }
    return out;
  }

  // y = (A u - B^T p [+ AL]) , w_p = B u  in TK (coupled operator)
  template <class TK>
  void coupled_apply(const TK* u, const TK* p, TK* yu, TK* yp, bool al) {
    ops::Bmul<TK>(c_, nrb_, u, yp, (TK)1, nullptr, (TK)0);
    TK* ex = nullptr;
    if (al && gamma_ > 0) {
      Engine<TK> ek(c_, o_, nrb_, st_);
      TK* y = static_cast<TK*>(c_->workspace(std::string("alk_y") + (sizeof(TK) == 4 ? "_f" : "_d"), np() * sizeof(TK)));
      ex = static_cast<TK*>(c_->workspace(std::string("alk_t") + (sizeof(TK) == 4 ? "_f" : "_d"), nu() * sizeof(TK)));
      ek.cheb_apply("alkq", c_->sQ, ops::pick<TK>(c_->MQ64, c_->MQ32), ops::pick<TK>(c_->dMQ64, c_->dMQ32), c_->bMQ,
                    std::is_same<TK, float>::value ? 18 : 26, nrb_, yp, y);
      ops::Btmul<TK>(c_, nrb_, y, nullptr, ex, (TK)(gamma_ * mu_), nullptr, (TK)0);
    }
    ops::momentum<TK>(c_, nrb_, u, p, ex, yu, (TK)1, nullptr);
  }

  // ------------------------------------------------------ FGMRES cycle
  // One restart cycle on K_gamma delta = r (Arnoldi basis and K_gamma in the
  // Krylov precision TK, preconditioner in T, Gram-Schmidt sums in FP64);
  // x += delta in FP64.  target[r]: absolute residual goal per right-hand side.
  int fgmres_cycle(const double* ru, const double* rp, double* xu, double* xp, const std::vector<double>& target,
                   int max_steps) {
    if constexpr (std::is_same<T, float>::value) {
      if (o_.arnoldi_fp64 == STOKES_ARNOLDI_FP32) return fgmres_cycle_t<float>(ru, rp, xu, xp, target, max_steps);
    }
    return fgmres_cycle_t<double>(ru, rp, xu, xp, target, max_steps);
  }

  template <class TK>
  int fgmres_cycle_t(const double* ru, const double* rp, double* xu, double* xp, const std::vector<double>& target,
                     int max_steps) {
    const int m = std::max(1, std::min({o_.restart, 63, max_steps}));
    const int64_t nc = nu() + np();
    const char* kt = std::is_same<TK, float>::value ? "_f" : "_d";
    TK* V = static_cast<TK*>(c_->workspace(std::string("gm_V") + kt, (m + 1) * nc * sizeof(TK)));
    T* Z = buf("gm_Z", m * nc);
    TK* w = static_cast<TK*>(c_->workspace(std::string("gm_w") + kt, nc * sizeof(TK)));
    const int nbx = ops::grid_for((c_->n_int + c_->n_p1) * nrb_);
    double* part = static_cast<double*>(
        c_->workspace("gm_part", (int64_t)((m + 1 + kMdotChunk - 1) / kMdotChunk) * nbx * kMdotChunk * 8 * sizeof(double)));
    double* hdev = static_cast<double*>(c_->workspace("gm_h", 3 * 64 * 8 * sizeof(double)));
    double* h1 = hdev;
    double* h2 = hdev + 64 * 8;
    double* nrm = hdev + 2 * 64 * 8;
    double* hhost = static_cast<double*>(c_->workspace_host("gm_hh", 3 * 64 * 8 * sizeof(double)));
    double* yhost = static_cast<double*>(c_->workspace_host("gm_yh", 64 * 8 * sizeof(double)));
    double* ydev = static_cast<double*>(c_->workspace("gm_y", 64 * 8 * sizeof(double)));

    auto mdot = [&](const TK* Vb, int nb, const auto* x, double* hout) {
      using TX = std::remove_const_t<std::remove_pointer_t<decltype(x)>>;
      dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
        constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
        hipLaunchKernelGGL((k_mdot<TK, TX, D, N>), dim3(nbx, (nb + kMdotChunk - 1) / kMdotChunk), dim3(kBlock), 0,
                           c_->stream, c_->n_int, c_->n_p1, Vb, nc, nb, x, part);
        ops::check_launch();
        hipLaunchKernelGGL((k_mdot_fin<N>), dim3(nb), dim3(kBlock), 0, c_->stream, nbx, (const double*)part, hout);
      });
      ops::check_launch();
      ops::count_bytes(c_, double(nc) * (nb * sizeof(TK) + sizeof(TX)));  // nb basis vectors and x
    };
    auto mupdate = [&](auto* Vb, int nb, const double* h, double sgn, auto* x, double* res,
                       const double* sig2 = nullptr, T* wf = nullptr) {
      using TV = std::remove_const_t<std::remove_pointer_t<decltype(Vb)>>;
      using TW = std::remove_pointer_t<decltype(x)>;
      dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
        constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
        if (res) {
          hipLaunchKernelGGL((k_mupdate<TV, TW, D, N, 1, T>), dim3(nbx), dim3(kBlock), 0, c_->stream, c_->n_int,
                             c_->n_p1, (const TV*)Vb, nc, nb, h, sgn, x, res, c_->red.partials.as<double>(), sig2,
                             wf);
          ops::check_launch();
          hipLaunchKernelGGL((k_finish<N>), dim3(1), dim3(kBlock), 0, c_->stream,
                             (const double*)c_->red.partials.as<double>(), nbx, (int)FIN_STORE, N, (Scalars*)nullptr,
                             1, 0, 0, res);
        } else {
          hipLaunchKernelGGL((k_mupdate<TV, TW, D, N, 0, T>), dim3(nbx), dim3(kBlock), 0, c_->stream, c_->n_int,
                             c_->n_p1, (const TV*)Vb, nc, nb, h, sgn, x, res, c_->red.partials.as<double>(), sig2,
                             wf);
        }
      });
      ops::check_launch();
      // nb basis vectors read, x read and written (and its copy in T written)
      ops::count_bytes(c_, double(nc) * (nb * sizeof(TV) + 2 * sizeof(TW) + (wf ? sizeof(T) : 0)));
    };
    // the preconditioner's input v_j in T: the basis itself, or a rounded
    // copy written by the scaling that forms v_j
    T* vin = std::is_same<T, TK>::value ? nullptr : buf("gm_vin", nc);
    auto scale_into = [&](const std::vector<double>& s, const TK* src, TK* dst) {
      Coef8 cs{};
      for (int r = 0; r < 8; ++r) cs.v[r] = r < nrb_ ? s[r] : 0;
      dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
        constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
        hipLaunchKernelGGL((k_scale_coupled<TK, D, N, T>), dim3(ops::grid_for(nc)), dim3(kBlock), 0, c_->stream,
                           c_->n_int, c_->n_p1, cs, src, dst, vin);
      });
      ops::check_launch();
      ops::count_bytes(c_, double(nc) * (2 * sizeof(TK) + (vin ? sizeof(T) : 0)));
    };

    // V_0 = r / ||r|| (read in place when (ru, rp) is one coupled vector)
    const TK* w0 = w;
    if constexpr (std::is_same<TK, double>::value) {
      if (rp == ru + nu()) {
        w0 = ru;
      } else {
        ops::copy_dev(c_, w, ru, nu() * sizeof(double));
        ops::copy_dev(c_, w + nu(), rp, np() * sizeof(double));
      }
    } else {
      ops::cast<double, float>(c_, nu(), ru, w);
      ops::cast<double, float>(c_, np(), rp, w + nu());
    }
    mdot(w0, 1, w0, h1);
    HIP_CHECK(hipMemcpyAsync(hhost, h1, nrb_ * sizeof(double), hipMemcpyDeviceToHost, c_->stream));
    HIP_CHECK(hipStreamSynchronize(c_->stream));
    const int R = nrb_;
    std::vector<double> beta(R), g((m + 1) * R, 0.0), H((m + 1) * m * R, 0.0), cs(m * R), sn(m * R);
    std::vector<int> active(R), kdone(R, 0);
    std::vector<double> s(R);
    for (int r = 0; r < R; ++r) {
      if (!std::isfinite(hhost[r])) throw Error(STOKES_ERR_NONFINITE, "FGMRES: non-finite residual norm");
      beta[r] = std::sqrt(std::max(0.0, hhost[r]));
      active[r] = beta[r] > target[r];
      s[r] = active[r] ? 1.0 / beta[r] : 0.0;
      g[0 * R + r] = beta[r];
    }
    scale_into(s, w0, V);
    // The basis after v_0 is kept unnormalized: column i holds v_i / sig[i]
    // (sig per right-hand side, on the host; its square on the device for
    // the Gram-Schmidt coefficients).  Each new column is left where the
    // second update writes it, which saves a scaling pass per step; the
    // Hessenberg entries, the norms and the solution coefficients carry sig.
    std::vector<double> sig((m + 1) * R, 0.0);
    double* sig2host = static_cast<double*>(c_->workspace_host("gm_s2h", 64 * 8 * sizeof(double)));
    double* sig2dev = static_cast<double*>(c_->workspace("gm_s2", 64 * 8 * sizeof(double)));
    for (int r = 0; r < R; ++r) {
      sig[r] = active[r] ? 1.0 : 0.0;
      sig2host[r] = sig[r];
    }
    HIP_CHECK(hipMemcpyAsync(sig2dev, sig2host, R * sizeof(double), hipMemcpyHostToDevice, c_->stream));
    // Gram matrix of the stored columns for the one-update CGS2 (steps with
    // at most kFusedMax columns): column 0 is stored normalized
    const bool gram = c_->gram_cgs2 != 0;
    double* Rg = nullptr;
    double* hsum = nullptr;
    if (gram) {
      Rg = static_cast<double*>(c_->workspace("gm_R", (size_t)kGramLd * kGramLd * 8 * sizeof(double)));
      hsum = static_cast<double*>(c_->workspace("gm_hs", 64 * 8 * sizeof(double)));
      double* onesh = static_cast<double*>(c_->workspace_host("gm_R00", 8 * sizeof(double)));
      for (int r = 0; r < 8; ++r) onesh[r] = 1.0;
      HIP_CHECK(hipMemcpyAsync(Rg, onesh, 8 * sizeof(double), hipMemcpyHostToDevice, c_->stream));
    }
    auto Hat = [&](int i, int j, int r) -> double& { return H[((size_t)i * m + j) * R + r]; };
    // K_gamma z_j in the inner precision T (the FP32 matrices) unless the
    // FP64 operator is asked for
    const bool k_inner = std::is_same<T, TK>::value || o_.arnoldi_fp64 != STOKES_ARNOLDI_FP64_K;
    // with the upper triangular preconditioner the product B^T z_p of the
    // preconditioner is reused by K_gamma z_j
    const bool reuse_bt = k_inner && o_.coupled_pc == STOKES_PC_UPPER && gamma_ == 0;
    T* bt = reuse_bt ? buf("gm_bt", nu()) : nullptr;
    // z_jj = P^{-1} v_jj in the inner precision: its input is the basis
    // column itself, or the rounded copy vin that the step before wrote
    auto precondition = [&](int jj) {
      const T* vsrc;
      if constexpr (std::is_same<T, TK>::value) {
        vsrc = V + (int64_t)jj * nc;
      } else {
        vsrc = vin;
      }
      T* Zjj = Z + (int64_t)jj * nc;
      block_prec(vsrc, vsrc + nu(), Zjj, Zjj + nu(), bt);
    };
    // With one right-hand side far from its goal, the preconditioner of the
    // next step is queued before the host reads this step's Gram-Schmidt
    // sums (it needs no host value), so the GPU does not idle while the
    // host applies the rotations; the host waits on an event recorded
    // before it.  Near the goal the step may be the last one, and the host
    // waits for the stream as before.  A queued z past the last step is
    // left unused.
    hipEvent_t ev_h = nullptr;
    HIP_CHECK(hipEventCreateWithFlags(&ev_h, hipEventDisableTiming));
    struct EventGuard {
      hipEvent_t e;
      ~EventGuard() { (void)hipEventDestroy(e); }
    } ev_guard{ev_h};
    // only for a fixed preconditioner (FIXED inner mode: a linear map that
    // accepts any input; TOL-mode inner CGs stop with an error on a
    // vanishing right-hand side, which a step past convergence can be)
    const bool queue_ahead = R == 1 && o_.inner_mode == STOKES_INNER_FIXED;
    bool z_queued = false;             // z_j already queued during step j - 1
    double est_prev = g[0];            // residual estimate after the previous step (R = 1)
    std::vector<double> last_est(beta);  // per right-hand side, for the residual history
    int j = 0;
    for (; j < m; ++j) {
      bool any = false;
      for (int r = 0; r < R; ++r) any = any || active[r];
      if (!any) break;
      T* Zj = Z + (int64_t)j * nc;
      TK* wj = V + (int64_t)(j + 1) * nc;  // K_gamma z_j, orthogonalized in place: the next column
      if (!z_queued) precondition(j);
      z_queued = false;
      // w = K_gamma z_j
      auto k_apply_inner = [&](T* out) {
        if (reuse_bt) {
          ops::velop<T>(c_, nrb_, Zj, out, (T)1, bt, (T)-1);             // A z_u - B^T z_p
          ops::Bmul<T>(c_, nrb_, Zj, out + nu(), (T)1, nullptr, (T)0);  // B z_u
        } else {
          coupled_apply<T>(Zj, Zj + nu(), out, out + nu(), true);
        }
      };
      T* wk = nullptr;  // K_gamma z_j in T, read by the first Gram-Schmidt pass
      if constexpr (std::is_same<T, TK>::value) {
        k_apply_inner(wj);
      } else if (k_inner) {
        wk = buf("gm_wk", nc);
        k_apply_inner(wk);
        if (j + 1 > kFusedMax) {
          ops::cast<T, TK>(c_, nc, wk, wj);
          wk = nullptr;
        }
      } else {
        TK* zk = static_cast<TK*>(c_->workspace(std::string("gm_zk") + kt, nc * sizeof(TK)));
        ops::cast<T, TK>(c_, nc, Zj, zk);
        coupled_apply<TK>(zk, zk + nu(), wj, wj + nu(), true);
      }
      // CGS2 (the first update and the second projection share one pass
      // over the basis while it holds at most kFusedMax vectors)
      const double t0 = now();
      const bool orth_timed = ops::phase_begin(c_, PHASE_ORTH);
      if (wk) mdot(V, j + 1, (const T*)wk, h1);
      else mdot(V, j + 1, (const TK*)wj, h1);
      if (gram && j + 1 <= kFusedMax) {
        // CGS2 in one update: the second projection's dots from the Gram
        // matrix, then w <- w - V s^2 (h1 + h2), which also writes the next
        // preconditioner input and the new column's Gram row and norm
        dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
          constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
          hipLaunchKernelGGL((k_gram_h2<N>), dim3(1), dim3(kBlock), 0, c_->stream, j + 1, (const double*)Rg,
                             (const double*)sig2dev, (const double*)h1, h2, hsum);
          ops::check_launch();
          auto go = [&](auto NMc) {
            constexpr int NM = decltype(NMc)::value;
            if (wk)
              hipLaunchKernelGGL((k_mupdate_dot<TK, TK, D, N, T, 1, T, NM>), dim3(nbx), dim3(kBlock), 0, c_->stream,
                                 c_->n_int, c_->n_p1, (const TK*)V, nc, j + 1, (const double*)hsum, (const T*)wk, wj,
                                 part, (const double*)sig2dev, vin);
            else
              hipLaunchKernelGGL((k_mupdate_dot<TK, TK, D, N, TK, 1, T, NM>), dim3(nbx), dim3(kBlock), 0, c_->stream,
                                 c_->n_int, c_->n_p1, (const TK*)V, nc, j + 1, (const double*)hsum, (const TK*)wj, wj,
                                 part, (const double*)sig2dev, vin);
          };
          if (j + 1 <= 8) go(std::integral_constant<int, 8>{});
          else go(std::integral_constant<int, kFusedMax>{});
          ops::check_launch();
          hipLaunchKernelGGL((k_gram_fin<N>), dim3(j + 2), dim3(kBlock), 0, c_->stream, nbx, (const double*)part, j + 1,
                             Rg, nrm);
        });
        ops::check_launch();
        // j + 1 basis vectors read once; w_j (or its T copy) read; the next column (and its T copy) written
        ops::count_bytes(c_, double(nc) * ((j + 1) * sizeof(TK) + (wk ? sizeof(T) : sizeof(TK)) + sizeof(TK) +
                                           (vin ? sizeof(T) : 0)));
      } else if (j + 1 <= kFusedMax) {
        dispatch_dn(D_, nrb_, [&](auto Dc, auto Nc) {
          constexpr int D = decltype(Dc)::value, N = decltype(Nc)::value;
          auto go = [&](auto NMc) {
            constexpr int NM = decltype(NMc)::value;
            if (wk)
              hipLaunchKernelGGL((k_mupdate_dot<TK, TK, D, N, T, 0, TK, NM>), dim3(nbx), dim3(kBlock), 0, c_->stream,
                                 c_->n_int, c_->n_p1, (const TK*)V, nc, j + 1, (const double*)h1, (const T*)wk, wj,
                                 part, (const double*)sig2dev, (TK*)nullptr);
            else
              hipLaunchKernelGGL((k_mupdate_dot<TK, TK, D, N, TK, 0, TK, NM>), dim3(nbx), dim3(kBlock), 0, c_->stream,
                                 c_->n_int, c_->n_p1, (const TK*)V, nc, j + 1, (const double*)h1, (const TK*)wj, wj,
                                 part, (const double*)sig2dev, (TK*)nullptr);
          };
          if (j + 1 <= 8) go(std::integral_constant<int, 8>{});
          else go(std::integral_constant<int, kFusedMax>{});
          ops::check_launch();
          hipLaunchKernelGGL((k_mdot_fin<N>), dim3(j + 1), dim3(kBlock), 0, c_->stream, nbx, (const double*)part, h2);
        });
        ops::check_launch();
        // j + 1 basis vectors read once for the update and the dots; w_j (or its T copy) read, w_j written
        ops::count_bytes(c_, double(nc) * ((j + 1) * sizeof(TK) + (wk ? sizeof(T) : sizeof(TK)) + sizeof(TK)));
      } else {
        mupdate(V, j + 1, h1, -1.0, wj, nullptr, sig2dev);
        mdot(V, j + 1, wj, h2);
      }
      // the second update also leaves the next preconditioner input (in T)
      if (!(gram && j + 1 <= kFusedMax)) mupdate(V, j + 1, h2, -1.0, wj, nrm, sig2dev, vin);
      if (orth_timed) ops::phase_end(c_, PHASE_ORTH);
      HIP_CHECK(hipMemcpyAsync(hhost, hdev, 3 * 64 * 8 * sizeof(double), hipMemcpyDeviceToHost, c_->stream));
      if (queue_ahead && j + 1 < m && est_prev > kQueueAhead * target[0]) {
        HIP_CHECK(hipEventRecord(ev_h, c_->stream));
        precondition(j + 1);
        z_queued = true;
        HIP_CHECK(hipEventSynchronize(ev_h));
      } else {
        HIP_CHECK(hipStreamSynchronize(c_->stream));
      }
      st_.seconds_orth += now() - t0;
      bool dropped = false;  // a right-hand side stopped while others go on
      for (int r = 0; r < R; ++r) {
        if (!active[r]) {
          s[r] = 0;
          continue;
        }
        const double sj = sig[j * R + r];
        for (int i = 0; i <= j; ++i)
          Hat(i, j, r) = sj * sig[i * R + r] * (hhost[i * R + r] + hhost[64 * 8 + i * R + r]);
        if (!std::isfinite(hhost[2 * 64 * 8 + r]) || !std::isfinite(hhost[r]) || !std::isfinite(hhost[64 * 8 + r]))
          throw Error(STOKES_ERR_NONFINITE, "FGMRES: non-finite Gram-Schmidt sums at step " + std::to_string(j));
        const double wn = std::sqrt(std::max(0.0, hhost[2 * 64 * 8 + r]));
        const double hn = sj * wn;
        if (log_level() >= 2) {
          double hs = hn * hn;
          for (int i = 0; i <= j; ++i) hs += Hat(i, j, r) * Hat(i, j, r);
          std::fprintf(stderr, "[stokes] arnoldi j=%d r=%d |w_perp|/|w| = %.3e\n", j, r, hn / std::sqrt(hs));
        }
        // apply previous rotations, then a new one
        for (int i = 0; i < j; ++i) {
          const double a = Hat(i, j, r), b = Hat(i + 1, j, r);
          Hat(i, j, r) = cs[i * R + r] * a + sn[i * R + r] * b;
          Hat(i + 1, j, r) = -sn[i * R + r] * a + cs[i * R + r] * b;
        }
        const double a = Hat(j, j, r);
        const double den = std::hypot(a, hn);
        const double cc = den > 0 ? a / den : 1.0, ss = den > 0 ? hn / den : 0.0;
        cs[j * R + r] = cc;
        sn[j * R + r] = ss;
        Hat(j, j, r) = den;
        g[(j + 1) * R + r] = -ss * g[j * R + r];
        g[j * R + r] = cc * g[j * R + r];
        kdone[r] = j + 1;
        const double est = std::fabs(g[(j + 1) * R + r]);
        if (r == 0) est_prev = est;
        last_est[r] = est;
        if (est <= target[r] || hn <= 1e-300) active[r] = 0;
        s[r] = active[r] && wn > 0 ? 1.0 : 0.0;
        sig[(j + 1) * R + r] = active[r] && wn > 0 ? 1.0 / wn : 0.0;
        dropped = dropped || !active[r];
      }
      st_.outer += 1;
      record_hist(last_est);
      if (j + 1 < m) {
        bool any_left = false;
        for (int r = 0; r < R; ++r) any_left = any_left || active[r];
        // zero the finished right-hand sides' part of the new column (it
        // would otherwise grow unnormalized through the later steps)
        if (dropped && any_left) scale_into(s, wj, wj);
        for (int r = 0; r < R; ++r) sig2host[(j + 1) * R + r] = sig[(j + 1) * R + r] * sig[(j + 1) * R + r];
        HIP_CHECK(hipMemcpyAsync(sig2dev + (j + 1) * R, sig2host + (j + 1) * R, R * sizeof(double),
                                 hipMemcpyHostToDevice, c_->stream));
      }
    }
    // y = H^{-1} g per right-hand side; x += Z y
    const int steps = j;
    std::fill(yhost, yhost + 64 * 8, 0.0);
    for (int r = 0; r < R; ++r) {
      const int k = kdone[r];
      for (int i = k - 1; i >= 0; --i) {
        double acc = g[i * R + r];
        for (int l = i + 1; l < k; ++l) acc -= Hat(i, l, r) * yhost[l * R + r];
        yhost[i * R + r] = Hat(i, i, r) != 0 ? acc / Hat(i, i, r) : 0.0;
      }
    }
    if (steps > 0) {
      for (int i = 0; i < steps; ++i)
        for (int r = 0; r < R; ++r) yhost[i * R + r] *= sig[i * R + r];  // z_i = sig_i P(stored column i)
      HIP_CHECK(hipMemcpyAsync(ydev, yhost, steps * R * sizeof(double), hipMemcpyHostToDevice, c_->stream));
      // the update writes the coupled vector (xu, xp): in place when the two
      // parts are contiguous, else through a staging copy
      if (xp == xu + nu()) {
        mupdate((const T*)Z, steps, ydev, 1.0, xu, nullptr);
      } else {
        double* xc = static_cast<double*>(c_->workspace("gm_x", nc * sizeof(double)));
        ops::copy_dev(c_, xc, xu, nu() * sizeof(double));
        ops::copy_dev(c_, xc + nu(), xp, np() * sizeof(double));
        mupdate((const T*)Z, steps, ydev, 1.0, xc, nullptr);
        ops::copy_dev(c_, xu, xc, nu() * sizeof(double));
        ops::copy_dev(c_, xp, xc + nu(), np() * sizeof(double));
      }
      HIP_CHECK(hipStreamSynchronize(c_->stream));
    }
    return steps;
  }

  // ---------------------------------------------------- Schur FCG sweep
  // Correction (du, dp) of K_gamma (du, dp) = (ru, rp) by flexible CG on the
  // Schur complement; x += correction.  target: absolute continuity goal.
  int schur_sweep(const double* ru, const double* rp, double* xu, double* xp, const std::vector<double>& target,
                  int max_steps) {
    const int R = nrb_;
    T* tu = buf("sc_tu", nu());
    T* vu = buf("sc_vu", nu());
    T* tp = buf("sc_tp", np());
    T* zp = buf("sc_zp", np());
    double* s = static_cast<double*>(c_->workspace("sc_s", np() * sizeof(double)));
    double* z = static_cast<double*>(c_->workspace("sc_z", np() * sizeof(double)));
    double* zo = static_cast<double*>(c_->workspace("sc_zo", np() * sizeof(double)));
    double* pp = static_cast<double*>(c_->workspace("sc_p", np() * sizeof(double)));
    double* q = static_cast<double*>(c_->workspace("sc_q", np() * sizeof(double)));
    auto to_T = [&](const double* x, T* y, int64_t n) {
      if (std::is_same<T, double>::value) ops::copy_dev(c_, y, x, n * sizeof(T));
      else ops::cast<double, float>(c_, n, x, reinterpret_cast<float*>(y));
    };
    auto to_64 = [&](const T* x, double* y, int64_t n) {
      if (std::is_same<T, double>::value) ops::copy_dev(c_, y, x, n * sizeof(T));
      else ops::cast<float, double>(c_, n, reinterpret_cast<const float*>(x), y);
    };
    std::vector<double> one(R, 1.0), zero(R, 0.0), mone(R, -1.0);
    // w_u = A~^{-1} r_u ; x_u += w_u ; s = r_p - B w_u
    to_T(ru, tu, nu());
    vel_solve(tu, vu);
    axpy_rhs<T, double>(c_->n_int, true, one.data(), one.data(), vu, xu);
    ops::Bmul<T>(c_, nrb_, vu, tp, (T)1, nullptr, (T)0);
    to_64(tp, q, np());
    ops::copy_dev(c_, s, rp, np() * sizeof(double));
    ops::axpby<double>(c_, np(), -1.0, q, 1.0, s);
    ops::remove_mean<double>(c_, nrb_, s);
    auto cc64 = [&](const double* in, double* out) {
      to_T(in, tp, np());
      cc_apply(tp, zp);
      to_64(zp, out, np());
    };
    std::vector<double> ss = dots(nullptr, nullptr, s, s);
    std::vector<int> active(R);
    bool any = false;
    for (int r = 0; r < R; ++r) {
      active[r] = std::sqrt(ss[r]) > target[r];
      any = any || active[r];
    }
    if (!any) return 0;
    cc64(s, z);
    std::vector<double> rho = dots(nullptr, nullptr, s, z);
    ops::copy_dev(c_, pp, z, np() * sizeof(double));
    int it = 0;
    while (it < max_steps) {
      ++it;
      st_.outer += 1;
      // q = S p = B A~^{-1} B^T p
      to_T(pp, tp, np());
      ops::Btmul<T>(c_, nrb_, tp, nullptr, tu, (T)1, nullptr, (T)0);
      vel_solve(tu, vu);
      ops::Bmul<T>(c_, nrb_, vu, tp, (T)1, nullptr, (T)0);
      to_64(tp, q, np());
      std::vector<double> sig = dots(nullptr, nullptr, pp, q);
      std::vector<double> al(R, 0.0), mal(R, 0.0);
      for (int r = 0; r < R; ++r) {
        if (!active[r]) continue;
        if (!(sig[r] > 0)) throw Error(STOKES_ERR_BREAKDOWN, "Schur CG breakdown (non-positive curvature)");
        al[r] = rho[r] / sig[r];
        mal[r] = -al[r];
      }
      axpy_rhs<double, double>(c_->n_p1, false, al.data(), one.data(), pp, xp);
      axpy_rhs<T, double>(c_->n_int, true, al.data(), one.data(), vu, xu);
      axpy_rhs<double, double>(c_->n_p1, false, mal.data(), one.data(), q, s);
      ss = dots(nullptr, nullptr, s, s);
      {
        std::vector<double> sn(R);
        for (int r = 0; r < R; ++r) sn[r] = std::sqrt(std::max(0.0, ss[r]));
        record_hist(sn);
      }
      any = false;
      for (int r = 0; r < R; ++r) {
        if (active[r] && !(std::sqrt(ss[r]) > target[r])) active[r] = 0;
        any = any || active[r];
      }
      if (!any) break;
      std::swap(z, zo);
      cc64(s, z);
      std::vector<double> rz = dots(nullptr, nullptr, s, z);
      std::vector<double> rzo = dots(nullptr, nullptr, s, zo);
      std::vector<double> be(R, 0.0);
      for (int r = 0; r < R; ++r) {
        if (active[r] && rho[r] != 0) be[r] = (rz[r] - rzo[r]) / rho[r];  // Polak-Ribiere (flexible)
        rho[r] = rz[r];
      }
      axpy_rhs<double, double>(c_->n_p1, false, one.data(), be.data(), z, pp);
    }
    return it;
  }

 private:
  stokes_ctx* c_;
  stokes_solve_opts o_;
  int nrb_, D_, W_;
  SolveStats& st_;
  double gamma_, mu_, alpha_;
  int al_deg_, cc_mq_deg_, mv_deg_;
};

// ======================================================================
// Refinement loop: x (internal FP64) solves K x = b, b = (F, g).
template <class T>
int refine_loop(stokes_ctx* c, const stokes_solve_opts& o, int method, int nrb, const double* F, const double* g,
                double* xu, double* xp, SolveStats& st, bool x_zero) {
  Engine<T> e(c, o, nrb, st);
  Engine<double> e64(c, o, nrb, st);
  const int64_t nu = c->n_int * c->dim * nrb, np = c->n_p1 * nrb;
  // (ru, rp) contiguous: the FGMRES cycle normalizes the coupled residual in place
  double* ru = static_cast<double*>(c->workspace("rf_r", (nu + np) * sizeof(double)));
  double* rp = ru + nu;
  std::vector<double> bn = e64.dots(F, F, g, g);
  for (double& x : bn) x = std::sqrt(x);
  for (int r = 0; r < nrb; ++r)
    if (!std::isfinite(bn[r]))
      throw Error(STOKES_ERR_NONFINITE, "right-hand side " + std::to_string(r) +
                                            " is not finite (forcing, boundary data or loss gradient)");
  st.inv_bn.assign(nrb, 0.0);
  for (int r = 0; r < nrb; ++r) st.inv_bn[r] = bn[r] > 0 ? 1.0 / bn[r] : 0.0;
  st.rel_res.assign(nrb, 0.0);
  int status = STOKES_NOT_CONVERGED;
  std::vector<double> prev(nrb, 0.0);
  int stalls = 0;
  for (int sweep = 0;; ++sweep) {
    // r = b - K x (plain system, FP64); r = b while x is still zero
    if (sweep == 0 && x_zero) {
      ops::copy_dev(c, ru, F, nu * sizeof(double));
      ops::copy_dev(c, rp, g, np * sizeof(double));
    } else {
      ops::momentum<double>(c, nrb, xu, xp, nullptr, ru, -1.0, F);
      ops::Bmul<double>(c, nrb, xu, rp, -1.0, g, 1.0);
    }
    std::vector<double> rn = e64.dots(ru, ru, rp, rp);
    std::vector<double> target(nrb);
    bool done = true;
    for (int r = 0; r < nrb; ++r) {
      rn[r] = std::sqrt(rn[r]);
      if (!std::isfinite(rn[r]))
        throw Error(STOKES_ERR_NONFINITE, sweep == 0 && !x_zero
                                              ? "the residual of the initial guess is not finite"
                                              : "the solve produced a non-finite residual at refinement sweep " +
                                                    std::to_string(sweep));
      st.rel_res[r] = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
      if (bn[r] > 0 && st.rel_res[r] > o.rtol) done = false;
      // goal of this sweep: the final tolerance, or the reduction the inner
      // precision can deliver (an FP32 Arnoldi relation holds to about 1e-7;
      // with an FP64 basis the 1e-5 goal is kept too, since a restart after
      // half the steps makes the Gram-Schmidt sums of the cycle cheaper)
      const double floor_rel = method == 0 ? (std::is_same<T, float>::value ? 1e-5 : 0.0)
                                           : (std::is_same<T, float>::value ? std::max(10 * o.inner_rtol_u, 1e-5)
                                                                            : 10 * o.inner_rtol_u);
      target[r] = std::max(0.5 * o.rtol * bn[r], floor_rel * rn[r]);
    }
    if (log_level() >= 1) {
      double worst = 0;
      for (double v : st.rel_res) worst = std::max(worst, v);
      std::fprintf(stderr, "[stokes] sweep %d: max rel res %.3e (outer %d, inner u %d, p %d)\n", sweep, worst,
                   st.outer, st.inner_u, st.inner_p);
    }
    if (done) {
      status = STOKES_OK;
      break;
    }
    // stagnation: two sweeps in a row without a 10% reduction
    bool progress = sweep == 0;
    for (int r = 0; r < nrb; ++r) progress = progress || rn[r] < 0.9 * prev[r];
    stalls = progress ? 0 : stalls + 1;
    prev = rn;
    if (stalls >= 2 || sweep >= o.max_refine || st.outer >= o.max_outer) break;
    st.sweeps += 1;
    ops::remove_mean<double>(c, nrb, rp);
    if (c->prob.gamma > 0) {
      // right-hand side of the augmented system: r_u + gamma mu B^T M_Q^{-1} r_p.
      // A continuity error e left by the sweep returns in the plain momentum
      // residual as gamma mu B^T M_Q^{-1} e, so the sweep goal is divided by
      // the measured gain of that map.
      double* y = static_cast<double*>(c->workspace("rf_y", np * sizeof(double)));
      double* t = static_cast<double*>(c->workspace("rf_t", nu * sizeof(double)));
      e64.cheb_apply("rfq", c->sQ, c->MQ64.as<double>(), c->dMQ64.as<double>(), c->bMQ, 26, nrb, rp, y);
      ops::Btmul<double>(c, nrb, y, nullptr, t, c->prob.gamma * c->prob.mu, nullptr, 0.0);
      std::vector<double> tn = e64.dots(t, t, nullptr, nullptr);
      std::vector<double> pn = e64.dots(nullptr, nullptr, rp, rp);
      for (int r = 0; r < nrb; ++r)
        if (pn[r] > 0) target[r] /= 1.0 + std::sqrt(tn[r] / pn[r]);
      ops::axpby<double>(c, nu, 1.0, t, 1.0, ru);
    }
    const int budget = o.max_outer - st.outer;
    if (method == 0) e.fgmres_cycle(ru, rp, xu, xp, target, budget);
    else e.schur_sweep(ru, rp, xu, xp, target, budget);
  }
  ops::normalize_pressure<double>(c, nrb, xp);
  return status;
}

// ======================================================================
// One rotational incremental pressure-correction step, the comparator of
// Sec. 7.5 and Table 8: a momentum solve, then a pressure Poisson solve and a
// pressure-mass solve, each solved to a true FP64 relative residual <= rtol by inner CG
// in T with FP64 refinement:
//   A u = F + B^T p_old;   d = B u - g;   L_Q phi = -alpha d;   M_Q psi = d;
//   p = p_old + phi - mu psi, normalised to zero mean.
template <class T>
int projection_loop(stokes_ctx* c, const stokes_solve_opts& o, int nrb, const double* F, const double* g,
                    const double* pold, double* xu, double* xp, SolveStats& st) {
  stokes_solve_opts oi = o;
  const bool f32 = std::is_same<T, float>::value;
  const double inner = f32 ? std::max(o.rtol, 1e-5) : 0.5 * o.rtol;
  oi.inner_mode = STOKES_INNER_TOL;
  oi.inner_rtol_u = inner;
  oi.inner_rtol_p = inner;
  oi.schur_pc = STOKES_CC_LAPLACE;
  Engine<T> e(c, oi, nrb, st);
  e.no_augmented_lagrangian();
  Engine<double> e64(c, oi, nrb, st);
  const int64_t nu = c->n_int * c->dim * nrb, np = c->n_p1 * nrb;
  auto ws = [&](const char* name, int64_t n) { return static_cast<double*>(c->workspace(name, n * sizeof(double))); };
  T* rT = f32 ? e.buf("pj_rT", std::max(nu, np)) : nullptr;
  T* dT = f32 ? e.buf("pj_dT", std::max(nu, np)) : nullptr;
  double* r = ws("pj_r", std::max(nu, np));
  double* dd = ws("pj_dd", std::max(nu, np));
  double worst = 0;
  int status = STOKES_OK;
  // x = K^{-1} b to rtol: r = b - K x in FP64, inner solve in T, x += d.
  // negligible: per right-hand side, a right-hand side norm at the rounding
  // level of the data it was formed from (then x = 0).
  auto refined = [&](bool vel, bool mean_free, const double* b, double* x, auto apply64, auto innerT,
                     const std::vector<double>& negligible) {
    const int64_t n = vel ? nu : np;
    ops::zero_dev(c, x, n * sizeof(double));
    std::vector<double> bn = vel ? e64.dots(b, b, nullptr, nullptr) : e64.dots(nullptr, nullptr, b, b);
    for (int k = 0; k < nrb; ++k)
      if (!std::isfinite(bn[k]))
        throw Error(STOKES_ERR_NONFINITE, std::string("pressure-correction step: non-finite ") +
                                              (vel ? "velocity" : "pressure") + " right-hand side");
    bool skip = true;
    for (int k = 0; k < nrb; ++k) skip = skip && std::sqrt(bn[k]) <= negligible[k];
    if (skip) return;
    double rel = 0;
    for (int sweep = 0;; ++sweep) {
      apply64(x, r);
      ops::axpby<double>(c, n, 1.0, b, -1.0, r);  // r = b - K x
      std::vector<double> rn = vel ? e64.dots(r, r, nullptr, nullptr) : e64.dots(nullptr, nullptr, r, r);
      rel = 0;
      for (int k = 0; k < nrb; ++k) {
        if (!std::isfinite(rn[k]))
          throw Error(STOKES_ERR_NONFINITE, "pressure-correction step: non-finite residual");
        rel = std::max(rel, bn[k] > 0 ? std::sqrt(rn[k] / bn[k]) : 0.0);
      }
      if (rel <= o.rtol) break;
      if (mean_free) ops::remove_mean<double>(c, nrb, r);  // the pressure Laplacian acts on 1-perp
      if (sweep >= o.max_refine) {
        status = STOKES_NOT_CONVERGED;
        break;
      }
      st.sweeps += 1;
      if constexpr (std::is_same<T, double>::value) {
        innerT(r, dd);
      } else {
        ops::cast<double, T>(c, n, r, rT);
        innerT(rT, dT);
        ops::cast<T, double>(c, n, dT, dd);
      }
      ops::axpby<double>(c, n, 1.0, dd, 1.0, x);
    }
    worst = std::max(worst, rel);
  };
  // 1. velocity
  double* bu = ws("pj_bu", nu);
  if (pold) ops::Btmul<double>(c, nrb, pold, nullptr, bu, 1.0, F, 1.0);
  else ops::copy_dev(c, bu, F, nu * sizeof(double));
  refined(true, false, bu, xu, [&](const double* x, double* y) { ops::velop<double>(c, nrb, x, y, 1.0, nullptr, 0.0); },
          [&](const T* rr, T* z) { e.vel_solve(rr, z); }, std::vector<double>(nrb, 0.0));
  // 2. divergence data d = B u - g and the pressure Laplacian; d below
  // 1e-13 |B|_F |u| + 1e-12 |g| is cancellation noise (u already discretely
  // divergence free: the fixed point) and gives phi = psi = 0
  double* d = ws("pj_d", np);
  ops::Bmul<double>(c, nrb, xu, d, 1.0, g, -1.0);
  const double bfro = std::sqrt(ops::dot_host<double>(c, c->sB.nnz_pad * c->dim, 1, c->B64.as<double>(),
                                                      c->B64.as<double>())[0]);
  std::vector<double> un = e64.dots(xu, xu, nullptr, nullptr), gn = e64.dots(nullptr, nullptr, g, g);
  std::vector<double> neg_d(nrb), neg_phi(nrb);
  for (int k = 0; k < nrb; ++k) {
    neg_d[k] = 1e-13 * bfro * std::sqrt(un[k]) + 1e-12 * std::sqrt(gn[k]);
    neg_phi[k] = c->prob.alpha * neg_d[k];
  }
  double* bphi = ws("pj_bphi", np);
  ops::axpby<double>(c, np, -c->prob.alpha, d, 0.0, bphi);
  double* phi = ws("pj_phi", np);
  refined(false, true, bphi, phi,
          [&](const double* x, double* y) { ops::spmv<double>(c, c->sQ, c->LQ64.as<double>(), nrb, x, y, 1.0, nullptr, 0.0); },
          [&](const T* rr, T* z) {
            ops::PhaseScope phase(c, PHASE_PRES);
            e.x_solve(rr, z);
          },
          neg_phi);
  // 3. pressure mass
  double* psi = ws("pj_psi", np);
  refined(false, false, d, psi,
          [&](const double* x, double* y) { ops::spmv<double>(c, c->sQ, c->MQ64.as<double>(), nrb, x, y, 1.0, nullptr, 0.0); },
          [&](const T* rr, T* z) {
            ops::PhaseScope phase(c, PHASE_PRES);
            e.mq_solve(rr, z);
          },
          neg_d);
  // 4. p = p_old + phi - mu psi
  if (pold) ops::copy_dev(c, xp, pold, np * sizeof(double));
  else ops::zero_dev(c, xp, np * sizeof(double));
  ops::axpby<double>(c, np, 1.0, phi, 1.0, xp);
  ops::axpby<double>(c, np, -c->prob.mu, psi, 1.0, xp);
  ops::normalize_pressure<double>(c, nrb, xp);
  st.rel_res.assign(nrb, worst);
  return status;
}

int projection_internal(stokes_ctx* c, const stokes_solve_opts& o, int nrb, const double* F, const double* g,
                        const double* pold, double* xu, double* xp, SolveStats& st) {
  if (o.vel_pc == STOKES_VEL_MG && c->mesh.order == 3)
    throw Error(STOKES_ERR_UNSUPPORTED, "the velocity multigrid needs the P2/P1 pair");
  ops::ensure_lanes(c, c->dim * nrb, false);
  if (o.precision == STOKES_MIXED) ops::ensure_lanes(c, c->dim * nrb, true);
  if (o.vel_pc == STOKES_VEL_MG && (!c->vmg_built || c->vmg_mu != c->prob.mu)) build_vmg(c);
  if (o.precision == STOKES_MIXED) return projection_loop<float>(c, o, nrb, F, g, pold, xu, xp, st);
  return projection_loop<double>(c, o, nrb, F, g, pold, xu, xp, st);
}

template <class T>
void vel_cheb_apply(stokes_ctx* c, int nrb, int degree, const T* r, T* z) {
  stokes_solve_opts o;
  stokes_default_opts(&o);
  SolveStats st;
  Engine<T> e(c, o, nrb, st);
  e.cheb_apply("vfx", c->sA, ops::pick<T>(c->A64, c->A32), ops::pick<T>(c->dA64, c->dA32), c->bA, degree,
               c->dim * nrb, r, z);
}
template void vel_cheb_apply<float>(stokes_ctx*, int, int, const float*, float*);
template void vel_cheb_apply<double>(stokes_ctx*, int, int, const double*, double*);

int solve_internal(stokes_ctx* c, const stokes_solve_opts& o, int method, int nrb, const double* F, const double* g,
                   double* xu, double* xp, SolveStats& st, bool x_zero) {
  if (o.vel_pc == STOKES_VEL_MG && c->mesh.order == 3)
    throw Error(STOKES_ERR_UNSUPPORTED, "the velocity multigrid needs the P2/P1 pair");
  ops::ensure_lanes(c, c->dim * nrb, false);  // FP64 outer operator
  if (o.vel_pc == STOKES_VEL_MG && (!c->vmg_built || c->vmg_mu != c->prob.mu)) build_vmg(c);
  if (o.precision == STOKES_MIXED) ops::ensure_lanes(c, c->dim * nrb, true);
  if (o.precision == STOKES_MIXED) return refine_loop<float>(c, o, method, nrb, F, g, xu, xp, st, x_zero);
  return refine_loop<double>(c, o, method, nrb, F, g, xu, xp, st, x_zero);
}

}  // namespace stokes

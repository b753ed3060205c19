// Host-side launchers of the device kernels (dispatch over value type, the
// number of values per row W and (dim, right-hand sides per batch)).
#pragma once

#include <vector>

#include "common.h"

namespace stokes {

struct QSum;  // closing step of a deferred Chebyshev sum (kernels.h)

void assemble_ctx(stokes_ctx* c);
void assemble_p1(stokes_ctx* c, const HostMesh& m, MgLevel& L);
void build_mg(stokes_ctx* c);
void build_interleaved(stokes_ctx* c);  // interleaved copies for the bfloat16 Chebyshev steps and K_gamma
// Galerkin hierarchy on B_I Lambda_V^-1 B_I^T + M_Q (levels only; the dense
// coarsest inverse is added by build_mg)
void assemble_galerkin(stokes_ctx* c, MgHier& H);
// e = one multigrid V-cycle of hierarchy H applied to r (pressure layout)
template <class T>
void mg_vcycle(stokes_ctx* c, const MgHier& H, int nrb, const T* r, T* e, int level = 0);
// velocity multigrid: coarse level assembly, hierarchy build, one V-cycle of
// alpha M + mu L applied to W = dim x nrhs interleaved components
void assemble_p2_level(stokes_ctx* c, const HostMesh& m, VmgLevel& L);
void build_vmg(stokes_ctx* c);
template <class T>
void vel_vcycle(stokes_ctx* c, int W, const T* r, T* e, int level = 0);
void estimate_bounds(stokes_ctx* c);
void reform_A(stokes_ctx* c);
void lanczos_bounds(stokes_ctx* c, const Sell& S, const double* vals, const double* dinv, int steps, double& rlo,
                    double& rhi, double& gersh);

namespace ops {

int grid_for(int64_t rows);
// lanes per row of the velocity-row kernels, autotuned once per (W, precision)
void ensure_lanes(stokes_ctx* c, int W, bool f32);
bool prof_begin(stokes_ctx* c, const Sell* S, const void* vals, const void* avals);
void prof_end(stokes_ctx* c, double bytes);
// Phase timing (PHASE_*, opts.profile = 2): begin returns false when it is off or the
// stream is being captured; collect synchronises and returns the summed
// seconds of the recorded pairs, which it releases for reuse.
bool phase_begin(stokes_ctx* c, int k);
void phase_end(stokes_ctx* c, int k) noexcept;
double phase_collect(stokes_ctx* c, int k);
struct PhaseScope {
  stokes_ctx* c;
  int k;
  bool on;
  PhaseScope(stokes_ctx* cc, int kk) : c(cc), k(kk), on(phase_begin(cc, kk)) {}
  ~PhaseScope() {
    if (on) phase_end(c, k);
  }
};
void check_launch();

// Algorithmic bytes (stokes_solve_info::bytes_alg): every launcher adds what
// its kernel must move at least: the stored operator once (values of every
// padded entry, `planes` of them, and the index structure it reads), each
// streamed vector once per pass and each gathered vector once.
inline void count_bytes(stokes_ctx* c, double b) { c->abytes += b; }
inline double op_bytes(const Sell& S, double value_size, bool affine = true) {
  return double(S.nnz_pad) * S.planes * value_size + (affine ? S.idx_bytes_af : S.idx_bytes);
}
// stream-ordered device copy and zero fill, counted
inline void copy_dev(stokes_ctx* c, void* dst, const void* src, size_t bytes) {
  HIP_CHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  count_bytes(c, 2.0 * double(bytes));
}
inline void zero_dev(stokes_ctx* c, void* dst, size_t bytes) {
  HIP_CHECK(hipMemsetAsync(dst, 0, bytes, c->stream));
  count_bytes(c, double(bytes));
}

template <class T> const T* pick(const DevBuf& b64, const DevBuf& b32);

// y = a * (S x) + b * yin, S scalar SELL shared by W values per row
template <class T>
void spmv(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* x, T* y, T a, const T* yin, T b);
// p = a * B u + b * pin
template <class T>
void Bmul(stokes_ctx* c, int nrb, const T* u, T* p, T a, const T* pin, T b);
// u = a * scale .* (B^T p) + b * uin; btout (optional) = a * scale .* (B^T p)
template <class T>
void Btmul(stokes_ctx* c, int nrb, const T* p, const T* scale, T* u, T a, const T* uin, T b, T* btout = nullptr);
// y = a * (A x) + b * yin with the velocity operator (vector Laplacian block
// or, for strain contexts, the coupled alpha M + mu (L + D) blocks)
template <class T>
void velop(stokes_ctx* c, int nrb, const T* x, T* y, T a, const T* yin, T b);
// y = sgn (A u - B^T p + extra) + yin
template <class T>
void momentum(stokes_ctx* c, int nrb, const T* u, const T* p, const T* extra, T* y, T sgn, const T* yin);

// slot sums of x .* y (y null => x .* x), rw optional row weights
template <class T>
void dot_dev(stokes_ctx* c, int64_t nrows, int W, const T* x, const T* y, const double* rw, double* res);
template <class T>
std::vector<double> dot_host(stokes_ctx* c, int64_t nrows, int W, const T* x, const T* y, const double* rw = nullptr);

// x[row][r] -= mean over rows (l2 mean per right-hand side)
template <class T>
void remove_mean(stokes_ctx* c, int nrb, T* x);
template <class T>
void remove_mean_into(stokes_ctx* c, int nrb, const T* x, T* y);  // y = x - mean(x) per right-hand side
// x[row][r] -= (m . x_r) / (m . 1) with m = M_Q 1 (zero pressure integral)
template <class T>
void normalize_pressure(stokes_ctx* c, int nrb, T* x);

template <class Tin, class Tout>
void cast(stokes_ctx* c, int64_t n, const Tin* x, Tout* y);
template <class T>
void axpby(stokes_ctx* c, int64_t n, T a, const T* x, T b, T* y);
template <class T>
void axpy_sys(stokes_ctx* c, int64_t n, int W, int cps, const double* coef, double scale, const T* v, T* y);

// CG / Chebyshev building blocks (see kernels.h)
template <class T>
void cg_spmv(stokes_ctx* c, int64_t nrows, const Sell* S, const T* vals, int W, const T* z, const T* extra, T* q,
             T* p, Scalars* sc, int cps, int nsys);
template <class T>
void cg_update(stokes_ctx* c, int64_t nrows, int W, int prec, T* x, T* r, const T* p, const T* q, const T* dinv,
               T theta_inv, T* d0, T* z, Scalars* sc, int cps, int nsys);
template <class T>
void cheb_init(stokes_ctx* c, int64_t nrows, int W, const T* r, const T* dinv, T theta_inv, T* d0, T* z);
// first Chebyshev step from x0 = 0 with the prologue fused (writes d1, res, z)
template <class T>
void cheb_first(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* r, const T* dinv, T theta_inv, T* d1,
                T* res, T* z, T c1, T c2, int accumulate = 0);
template <class T>
void cheb_step(stokes_ctx* c, const Sell& S, const T* vals, int W, const T* d, T* dn, const T* res_in, T* res_out,
               T* z, const T* dinv, T c1, T c2, const T* rvec, Scalars* sc, int cps, int nsys, int first);
// The same operations on half-precision values scaled by 1/ms (S = ms x
// stored values), FP32 vectors: the pressure multigrid levels.
void spmv_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* x, float* y, float a,
             const float* yin, float b);
void cheb_first_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* r,
                   const float* dinv, float theta_inv, float* d1, float* res, float* z, float c1, float c2,
                   int accumulate);
void cheb_step_hs(stokes_ctx* c, const Sell& S, const _Float16* vals, float ms, int W, const float* d, float* dn,
                  const float* res_in, float* res_out, float* z, const float* dinv, float c1, float c2);
// The same with the direction q kept in bfloat16 (W = 3 rows padded to 4).
// zw = false: the deferred form, which leaves z to a closing step; fin: that
// closing step (res and qn are not stored, z = dinv (theta_inv r + q_1 + ...)).
void cheb_first_hb(stokes_ctx* c, int W, const float* r, const float* dinv, float theta_inv, uint16_t* q1,
                   float* res, float* z, float c1, float c2, bool zw = true);
void cheb_step_hb(stokes_ctx* c, int W, const uint16_t* q, uint16_t* qn, const float* res_in, float* res_out,
                  float* z, const float* dinv, float c1, float c2, const QSum* fin = nullptr, bool zw = true);
// The same two steps on the half-precision column-scaled velocity block
// A_II D^{-1} (ctx AD16) in the rescaled direction q = D d (FP32 vectors).
void cheb_first_h(stokes_ctx* c, int W, const float* r, const float* dinv, float theta_inv, float* q1, float* res,
                  float* z, float c1, float c2);
void cheb_step_h(stokes_ctx* c, int W, const float* q, float* qn, const float* res_in, float* res_out, float* z,
                 const float* dinv, float c1, float c2);

// layout transfers
template <class T>
void vel_in(stokes_ctx* c, int nrb, const double* src, T* dst);
template <class T>
void vel_out(stokes_ctx* c, int nrb, const T* src, const double* ubc, double* dst, int bnd_fill);
template <class T>
void p_in(stokes_ctx* c, int nrb, const double* src, T* dst);
template <class T>
void p_out(stokes_ctx* c, int nrb, const T* src, double* dst);

// FP64 right-hand side and adjoint gradient pieces
// fI: staging buffer of n_int * dim * nrb doubles for the interior forcing
// (nullptr: a context workspace)
void rhs(stokes_ctx* c, int nrb, const double* f, const double* ubc, double* F, double* g, double* fI = nullptr);
void adj_jp(stokes_ctx* c, int nrb, double* g);
void adj_dJdf(stokes_ctx* c, int nrb, const double* lam, double* out);
void adj_dJdmu(stokes_ctx* c, int nrb, const double* u_full, const double* lam, double* res_dev);

}  // namespace ops
}  // namespace stokes

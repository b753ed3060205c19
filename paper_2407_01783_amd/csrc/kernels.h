// Device kernels of the solver: sliced-ELL SpMV/SpMM with fused Krylov
// epilogues, B / B^T, one-pass deterministic grid reductions, vector updates
// and layout conversions.  Everything here is memory-bandwidth bound; no MFMA.
//
// Vector layouts (internal):
//   velocity  T[n_int][nrb][dim]   (W = dim * nrb values per interior node)
//   pressure  T[n_p1][nrb]
// Reductions produce one partial per "slot" w < W (the value index inside a
// row); systems are groups of cps consecutive slots (cps = 1 for one CG per
// component and right-hand side, cps = dim for a joint vector CG).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"

namespace stokes {

__host__ __device__ inline int64_t ipow_dev(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Reduce v[0..NS) over the block; thread s < NS receives the block total of
// slot s in the return array `out` (shared).  Fixed order => deterministic.
template <int NS>
__device__ __forceinline__ void block_sum(double (&v)[NS], double* out_shared) {
  __shared__ double sh[kBlock / 64][NS];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double t = wave_sum(v[s]);
    if (lane == 0) sh[wid][s] = t;
  }
  __syncthreads();
  if (threadIdx.x < NS) {
    double a = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) a += sh[w][threadIdx.x];
    out_shared[threadIdx.x] = a;
  }
  __syncthreads();
}

// Block partials of a grid reduction: block b stores its NS slot sums at
// partials[b * NS + s].  A separate one-block kernel (k_finish) adds them in
// block order after the kernel boundary, so no device-scope fence is needed
// (a fence per block writes back the whole L2 on a multi-XCD part) and the
// result is deterministic.
template <int NS>
__device__ __forceinline__ void grid_reduce(double (&v)[NS], double* partials) {
  __shared__ double tot[NS];
  block_sum<NS>(v, tot);
  if (threadIdx.x < NS) partials[(size_t)blockIdx.x * NS + threadIdx.x] = tot[threadIdx.x];
}

enum FinKind { FIN_STORE = 0, FIN_ALPHA = 1, FIN_RR = 2, FIN_RR_RHO = 3, FIN_RHO = 4 };

// Sum the block partials (fixed order) and finish the Krylov scalars:
//   FIN_STORE   res[s] = total of slot s
//   FIN_ALPHA   sigma = p.q per system, alpha = rho / sigma (0 if inactive)
//   FIN_RR      rr = r.r per system, deactivate converged systems
//   FIN_RR_RHO  FIN_RR and rho = r.z (slots W..2W-1), beta = rho / rho_old
//   FIN_RHO     rho = r.z, beta = rho / rho_old (0 when `first`)
template <int NS>
__global__ __launch_bounds__(kBlock) void k_finish(const double* __restrict__ partials, int nblocks, int kind, int W,
                                                   Scalars* sc, int cps, int nsys, int first, double* res) {
  double a[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) a[s] = 0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int s = 0; s < NS; ++s) a[s] += partials[(size_t)b * NS + s];
  }
  __shared__ double tot[NS];
  block_sum<NS>(a, tot);
  const int s = threadIdx.x;
  if (kind == FIN_STORE) {
    if (s < NS) res[s] = tot[s];
    return;
  }
  if (s >= nsys) return;
  auto sum = [&](int off) {
    double x = 0;
    for (int w = s * cps; w < (s + 1) * cps; ++w) x += tot[off + w];
    return x;
  };
  if (kind == FIN_ALPHA) {
    const double sig = sum(0);
    sc->sigma[s] = sig;
    double al = 0;
    if (sc->active[s]) {
      if (sig > 0) al = sc->rho[s] / sig;
      else sc->breakdown = 1;
    }
    sc->alpha[s] = al;
    return;
  }
  if (kind == FIN_RR || kind == FIN_RR_RHO) {
    const double rr = sum(0);
    sc->rr[s] = rr;
    if (sc->active[s] && !(rr > sc->tol2[s])) sc->active[s] = 0;
  }
  if (kind == FIN_RR_RHO || kind == FIN_RHO) {
    const double rho = sum(kind == FIN_RR_RHO ? W : 0);
    if (first) sc->beta[s] = 0.0;
    else sc->beta[s] = (sc->active[s] && sc->rho[s] != 0) ? rho / sc->rho[s] : 0.0;
    if (sc->active[s] && !(rho > 0)) sc->breakdown = 1;
    sc->rho[s] = rho;
  }
}

// --------------------------------------------------------- SELL row sums
//
// Sliced ELL with slice height 64 (one wavefront): entry j of row r sits at
// sp[r / 64] + 64 j + (r mod 64), so the lanes of a wavefront read
// consecutive column indices and values.  Right-hand sides are interleaved:
// a velocity-shaped vector holds W = dim x nrhs values per row.
//
// G lanes per row (G in {1, 2, 4, 8}, dividing W): the lanes of a group walk
// the same row -- they load the same index and value, which the memory
// pipeline merges -- and each gathers and accumulates its own W / G
// consecutive components.  With large W this turns one wavefront-wide gather
// of 64 scattered W-vectors into a few contiguous segments per column; the
// summation order of every component is the same for every G.
//
// Column indices come in one of three forms per slice (SellIdx): computed
// (affine) -- slot j of lane l is base_j + l, plus a jump from a break lane
// on, from two words per slot that every lane reads alike (scalar loads) --;
// packed -- slot j of the slice holds a base column plus an 8-bit lane
// offset, so a lane reads one byte per entry -- or plain 32-bit columns
// where a slot spreads over more than 256 columns.  Every walker takes the
// computed form where the slice has it (the packed offsets stay valid for
// it too).  The rows of a wavefront always lie in one slice (an aligned
// group of 64 / G rows), so the slice index is read from the first active
// lane and the form is a uniform branch.
//
// Entries of a row are walked U at a time (U = 4; 8 when a lane carries two
// components, 16 when it carries one) so that 2U matrix loads and U W/G
// gathers are in flight per lane.
struct SliceRef {
  int64_t beg;  // entry 0 of the row
  int64_t eb;   // first slot of the slice (index into cbase)
  int width;    // slots of the slice
  bool pk;      // packed columns
  bool af;      // affine slots (columns computed from cmeta; packed offsets also valid)
  int pg;       // leading four-slot sub-groups made of two adjacent-node slot pairs (affine slices)
};

__device__ __forceinline__ SliceRef slice_ref(const SellIdx& ix, int64_t row) {
  const int64_t s = __builtin_amdgcn_readfirstlane(static_cast<int>(row >> 6));
  const int64_t s0 = ix.sp[s];
  SliceRef r;
  r.beg = s0 + (row & 63);
  r.eb = s0 >> 6;
  r.width = static_cast<int>((ix.sp[s + 1] - s0) >> 6);
  const int form = ix.pk[s];
  r.pk = form != 0;
  r.af = (form & 3) == 2 && ix.cmeta != nullptr;
  r.pg = r.af ? form >> 2 : 0;
  return r;
}

// Column of slot j of an affine slice: base + lane, plus the slot's jump from
// its break lane on (the two words of the slot are the same for every lane:
// scalar loads).  Meta word: break lane in bits 0-7 (0..64), jump from bit 8.
__device__ __forceinline__ int32_t affine_col(const SellIdx& ix, const SliceRef& r, int64_t slot) {
  const int lane = static_cast<int>(r.beg - (r.eb << 6));
  const int32_t base = ix.cmeta[2 * slot], meta = ix.cmeta[2 * slot + 1];
  return base + lane + (lane >= (meta & 0xFF) ? (meta >> 8) : 0);
}

// Column of slot j in form F: 0 = 32-bit columns, 1 = packed offsets,
// 2 = affine (computed).
template <int F>
__device__ __forceinline__ int32_t sell_col_f(const SellIdx& ix, const SliceRef& r, int j) {
  if constexpr (F == 2) return affine_col(ix, r, r.eb + j);
  else if constexpr (F == 1)
    return ix.cbase[r.eb + j] + static_cast<int32_t>(__builtin_nontemporal_load(ix.cdel + r.beg + 64 * j));
  else
    return __builtin_nontemporal_load(ix.cols + r.beg + 64 * j);
}

// acc += sum_j v_j x[c_j][sub W/G ...]; DS: v_j is multiplied by ds[c_j]
// Groups of U entries, then groups of 4 (U > 4) and single entries for the
// rest of the row, so short rows keep several loads in flight too.
template <typename T, int W, int G, typename TM, int F, bool DS, int U = 4>
__device__ __forceinline__ void sell_row_impl(const SellIdx& ix, const SliceRef& r, const TM* __restrict__ vals,
                                              const T* __restrict__ xs, const T* __restrict__ ds,
                                              T (&acc)[W / G]) {
  constexpr int WG = W / G;
  auto group = [&](auto Uc, int j) {
    constexpr int UU = decltype(Uc)::value;
    int32_t c[UU];
    T v[UU];
#pragma unroll
    for (int u = 0; u < UU; ++u) {
      c[u] = sell_col_f<F>(ix, r, j + u);
      v[u] = (T)__builtin_nontemporal_load(vals + r.beg + 64 * (j + u));
    }
    if constexpr (DS) {
#pragma unroll
      for (int u = 0; u < UU; ++u) v[u] *= ds[c[u]];
    }
    T xv[UU][WG];
#pragma unroll
    for (int u = 0; u < UU; ++u)
#pragma unroll
      for (int w = 0; w < WG; ++w) xv[u][w] = xs[(int64_t)c[u] * W + w];
#pragma unroll
    for (int u = 0; u < UU; ++u)
#pragma unroll
      for (int w = 0; w < WG; ++w) acc[w] = fma(v[u], xv[u][w], acc[w]);
  };
  int j = 0;
  for (; j + U <= r.width; j += U) group(std::integral_constant<int, U>{}, j);
  if constexpr (U > 4)
    for (; j + 4 <= r.width; j += 4) group(std::integral_constant<int, 4>{}, j);
  for (; j < r.width; ++j) group(std::integral_constant<int, 1>{}, j);
}

// TM is the storage type of the values (T, or _Float16 for a scaled copy);
// every product and sum runs in T.  ds (optional): column scaling of the
// values (S D), gathered at the columns.  U: entries per unrolled group.
template <typename T, int W, int G = 1, typename TM = T, int U = 4>
__device__ __forceinline__ void sell_row(const SellIdx& ix, const TM* __restrict__ vals, const T* __restrict__ x,
                                         int64_t row, int sub, T (&acc)[W / G], const T* __restrict__ ds = nullptr) {
  const SliceRef r = slice_ref(ix, row);
  const T* __restrict__ xs = x + sub * (W / G);
  if (ds) {
    if (r.af) sell_row_impl<T, W, G, TM, 2, true, U>(ix, r, vals, xs, ds, acc);
    else if (r.pk) sell_row_impl<T, W, G, TM, 1, true, U>(ix, r, vals, xs, ds, acc);
    else sell_row_impl<T, W, G, TM, 0, true, U>(ix, r, vals, xs, ds, acc);
  } else {
    if (r.af) sell_row_impl<T, W, G, TM, 2, false, U>(ix, r, vals, xs, ds, acc);
    else if (r.pk) sell_row_impl<T, W, G, TM, 1, false, U>(ix, r, vals, xs, ds, acc);
    else sell_row_impl<T, W, G, TM, 0, false, U>(ix, r, vals, xs, ds, acc);
  }
}

// ------------------------------------- interleaved SELL copies
//
// A copy of a slice's scalar arrays (values, packed column offsets, 32-bit
// columns) in which slots IW g .. IW g + IW - 1 of row r of a slice starting
// at entry s0 sit at s0 + 64 IW g + IW r + (0 .. IW - 1): one lane reads the
// IW values of a group with one load (16 bytes: IW = 4 for float values,
// 8 for half values) and their column offsets with one 4- or 8-byte load,
// where the slot-major layout takes one load per entry and array.  Slots
// from IW floor(width / IW) on keep their slot-major places (s0 + 64 j + r),
// so the copy is a permutation inside each slice with the same slice
// pointers and column bases (k_interleave).  Entries are still taken in slot
// order: products equal the slot-major ones bit for bit.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4a8_t __attribute__((ext_vector_type(4), aligned(8)));  // 16 bytes at 8-byte alignment

// slots per interleaved group for values of type TM
template <typename TM>
constexpr int il_width() {
  return sizeof(TM) == 2 ? 8 : 4;
}

__device__ __forceinline__ float half_bits(uint32_t h) {
  return (float)__builtin_bit_cast(_Float16, static_cast<uint16_t>(h));
}

// the IW values of a group (e = its first entry), as T
template <int IW, typename TM, typename T>
__device__ __forceinline__ void load_vals(const TM* __restrict__ vals, int64_t e, T (&v)[IW]) {
  static_assert(sizeof(TM) == 2 || sizeof(TM) == 4, "half or float values");
  if constexpr (sizeof(TM) == 2 && IW == 8) {
    const u32x4_t vv = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(vals + e));
    const uint32_t w[4] = {vv.x, vv.y, vv.z, vv.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = (T)half_bits(w[k] & 0xFFFFu);
      v[2 * k + 1] = (T)half_bits(w[k] >> 16);
    }
  } else if constexpr (sizeof(TM) == 2) {
    static_assert(IW == 4, "half groups of 4 or 8");
    const u32x2_t vv = __builtin_nontemporal_load(reinterpret_cast<const u32x2_t*>(vals + e));
    v[0] = (T)half_bits(vv.x & 0xFFFFu);
    v[1] = (T)half_bits(vv.x >> 16);
    v[2] = (T)half_bits(vv.y & 0xFFFFu);
    v[3] = (T)half_bits(vv.y >> 16);
  } else {
    static_assert(IW == 4, "float groups of 4");
    const f32x4_t vv = __builtin_nontemporal_load(reinterpret_cast<const f32x4_t*>(vals + e));
    v[0] = (T)vv.x;
    v[1] = (T)vv.y;
    v[2] = (T)vv.z;
    v[3] = (T)vv.w;
  }
}

// the IW columns of group g (e = its first entry), in form F (sell_col_f)
template <int IW, int F>
__device__ __forceinline__ void load_cols(const SellIdx& ix, const SliceRef& r, int g, int64_t e, int32_t (&c)[IW]) {
  static_assert(IW == 4 || IW == 8, "groups of 4 or 8");
  if constexpr (F == 2) {
#pragma unroll
    for (int k = 0; k < IW; ++k) c[k] = affine_col(ix, r, r.eb + IW * g + k);
  } else if constexpr (F == 1) {
    uint32_t d[IW / 4];
    if constexpr (IW == 4) {
      d[0] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(ix.cdel + e));
    } else {
      const u32x2_t dd = __builtin_nontemporal_load(reinterpret_cast<const u32x2_t*>(ix.cdel + e));
      d[0] = dd.x;
      d[1] = dd.y;
    }
#pragma unroll
    for (int k = 0; k < IW; ++k)
      c[k] = ix.cbase[r.eb + IW * g + k] + static_cast<int32_t>((d[k / 4] >> (8 * (k % 4))) & 0xFFu);
  } else {
#pragma unroll
    for (int q = 0; q < IW / 4; ++q) {
      const i32x4_t cc = __builtin_nontemporal_load(reinterpret_cast<const i32x4_t*>(ix.cols + e + 4 * q));
      c[4 * q] = cc.x;
      c[4 * q + 1] = cc.y;
      c[4 * q + 2] = cc.z;
      c[4 * q + 3] = cc.w;
    }
  }
}

// acc += sum_j v_j x[c_j][off .. off + W/G) over the interleaved copy (IW
// slots per group, il_width<TM>): G lanes per row, each taking W/G of the
// row's components (the lanes of a row read the same values and columns);
// eight entries in flight per lane.
template <typename T, int W, int G, typename TM, int F>
__device__ __forceinline__ void sell_row_il_impl(const SellIdx& ix, const SliceRef& r, const TM* __restrict__ vals,
                                                 const T* __restrict__ x, int off, T (&acc)[W / G]) {
  constexpr int WG = W / G, IW = il_width<TM>(), HG = 8 / IW;
  const int64_t s0 = r.eb << 6;
  const int lr = static_cast<int>(r.beg - s0);
  const int gi = r.width / IW;
  auto groups = [&](auto Hc, int g) {
    constexpr int H = decltype(Hc)::value;
    int32_t c[H][IW];
    T v[H][IW];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int64_t e = s0 + 64 * IW * (int64_t)(g + h) + IW * lr;
      load_vals<IW, TM, T>(vals, e, v[h]);
      load_cols<IW, F>(ix, r, g + h, e, c[h]);
    }
    T xv[H][IW][WG];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int k = 0; k < IW; ++k)
#pragma unroll
        for (int w = 0; w < WG; ++w) xv[h][k][w] = x[(int64_t)c[h][k] * W + off + w];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int k = 0; k < IW; ++k)
#pragma unroll
        for (int w = 0; w < WG; ++w) acc[w] = fma(v[h][k], xv[h][k][w], acc[w]);
  };
  int g = 0;
  for (; g + HG <= gi; g += HG) groups(std::integral_constant<int, HG>{}, g);
  // the last group (if any) and the width mod IW tail slots (slot-major) in
  // one round trip: every load first, then the sums in slot order
  const bool last = g < gi;
  const int t = r.width - IW * gi;
  if (!last && t == 0) return;
  int32_t c[IW], ct[IW - 1];
  T v[IW], vt[IW - 1];
  if (last) {
    const int64_t e = s0 + 64 * IW * (int64_t)g + IW * lr;
    load_vals<IW, TM, T>(vals, e, v);
    load_cols<IW, F>(ix, r, g, e, c);
  }
#pragma unroll
  for (int k = 0; k < IW - 1; ++k)
    if (k < t) {
      ct[k] = sell_col_f<F>(ix, r, IW * gi + k);
      vt[k] = (T)__builtin_nontemporal_load(vals + r.beg + 64 * (IW * gi + k));
    }
  T xv[IW][WG], xt[IW - 1][WG];
  if (last)
#pragma unroll
    for (int k = 0; k < IW; ++k)
#pragma unroll
      for (int w = 0; w < WG; ++w) xv[k][w] = x[(int64_t)c[k] * W + off + w];
#pragma unroll
  for (int k = 0; k < IW - 1; ++k)
    if (k < t)
#pragma unroll
      for (int w = 0; w < WG; ++w) xt[k][w] = x[(int64_t)ct[k] * W + off + w];
  if (last)
#pragma unroll
    for (int k = 0; k < IW; ++k)
#pragma unroll
      for (int w = 0; w < WG; ++w) acc[w] = fma(v[k], xv[k][w], acc[w]);
#pragma unroll
  for (int k = 0; k < IW - 1; ++k)
    if (k < t)
#pragma unroll
      for (int w = 0; w < WG; ++w) acc[w] = fma(vt[k], xt[k][w], acc[w]);
}

template <typename T, int W, int G, typename TM>
__device__ __forceinline__ void sell_row_il(const SellIdx& ix, const TM* __restrict__ vals, const T* __restrict__ x,
                                            int64_t row, int sub, T (&acc)[W / G]) {
  const SliceRef r = slice_ref(ix, row);
  const int off = sub * (W / G);
  if (r.af) sell_row_il_impl<T, W, G, TM, 2>(ix, r, vals, x, off, acc);
  else if (r.pk) sell_row_il_impl<T, W, G, TM, 1>(ix, r, vals, x, off, acc);
  else sell_row_il_impl<T, W, G, TM, 0>(ix, r, vals, x, off, acc);
}

// B rows (pressure vertex): acc[r] = sum_j sum_c B^c_j u[col_j][r][c]
// (entries walked two at a time to keep more loads in flight)
template <typename T, int D, int NRB, int F>
__device__ __forceinline__ void sell_row_B_impl(const SellIdx& ix, const SliceRef& rf, const T* __restrict__ vals,
                                                const T* __restrict__ u, T (&acc)[NRB]) {
  constexpr int U = 2;
  int j = 0;
  for (; j + U <= rf.width; j += U) {
    int32_t c[U];
    T b[U][D], x[U][D * NRB];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t k = rf.beg + 64 * (j + q);
      c[q] = sell_col_f<F>(ix, rf, j + q);
#pragma unroll
      for (int d = 0; d < D; ++d) b[q][d] = __builtin_nontemporal_load(vals + k * D + d);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < D * NRB; ++w) x[q][w] = u[(int64_t)c[q] * (D * NRB) + w];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int d = 0; d < D; ++d) acc[r] = fma(b[q][d], x[q][r * D + d], acc[r]);
  }
  for (; j < rf.width; ++j) {
    const int64_t k = rf.beg + 64 * j;
    const int32_t c = sell_col_f<F>(ix, rf, j);
    T b[D];
#pragma unroll
    for (int d = 0; d < D; ++d) b[d] = __builtin_nontemporal_load(vals + k * D + d);
    const T* up = u + (int64_t)c * (D * NRB);
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int d = 0; d < D; ++d) acc[r] = fma(b[d], up[r * D + d], acc[r]);
  }
}

template <typename T, int D, int NRB>
__device__ __forceinline__ void sell_row_B(const SellIdx& ix, const T* __restrict__ vals, const T* __restrict__ u,
                                           int64_t row, T (&acc)[NRB]) {
  const SliceRef rf = slice_ref(ix, row);
  if (rf.af) sell_row_B_impl<T, D, NRB, 2>(ix, rf, vals, u, acc);
  else if (rf.pk) sell_row_B_impl<T, D, NRB, 1>(ix, rf, vals, u, acc);
  else sell_row_B_impl<T, D, NRB, 0>(ix, rf, vals, u, acc);
}

// value plane d (runtime, d < D) of a small register array
template <typename T, int D>
__device__ __forceinline__ T plane(const T (&b)[D], int d) {
  T o = b[0];
#pragma unroll
  for (int e = 1; e < D; ++e) o = d == e ? b[e] : o;
  return o;
}

// B^T rows (interior velocity node): acc[r][c] = sum_j B^c_j p[col_j][r];
// with G lanes per row, lane `sub` owns components sub W/G .. (sub+1) W/G - 1
// of the W = D NRB outputs (component w is rhs w / D, plane w mod D).
template <typename T, int D, int NRB, int G, int F>
__device__ __forceinline__ void sell_row_Bt_impl(const SellIdx& ix, const SliceRef& rf, const T* __restrict__ vals,
                                                 const T* __restrict__ p, int sub, T (&acc)[D * NRB / G]) {
  constexpr int WG = D * NRB / G;
  int rr[WG], dd[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) {
    rr[w] = (sub * WG + w) / D;
    dd[w] = (sub * WG + w) - rr[w] * D;
  }
  constexpr int U = 4;
  int j = 0;
  for (; j + U <= rf.width; j += U) {
    int32_t c[U];
    T b[U][D], pv[U][WG];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t k = rf.beg + 64 * (j + q);
      c[q] = sell_col_f<F>(ix, rf, j + q);
#pragma unroll
      for (int d = 0; d < D; ++d) b[q][d] = __builtin_nontemporal_load(vals + k * D + d);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < WG; ++w) pv[q][w] = p[(int64_t)c[q] * NRB + rr[w]];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < WG; ++w) acc[w] = fma(G == 1 ? b[q][w % D] : plane<T, D>(b[q], dd[w]), pv[q][w], acc[w]);
  }
  for (; j < rf.width; ++j) {
    const int64_t k = rf.beg + 64 * j;
    const int32_t c = sell_col_f<F>(ix, rf, j);
    T b[D];
#pragma unroll
    for (int d = 0; d < D; ++d) b[d] = __builtin_nontemporal_load(vals + k * D + d);
    const T* pp = p + (int64_t)c * NRB;
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = fma(G == 1 ? b[w % D] : plane<T, D>(b, dd[w]), pp[rr[w]], acc[w]);
  }
}

template <typename T, int D, int NRB, int G = 1>
__device__ __forceinline__ void sell_row_Bt(const SellIdx& ix, const T* __restrict__ vals, const T* __restrict__ p,
                                            int64_t row, int sub, T (&acc)[D * NRB / G]) {
  const SliceRef rf = slice_ref(ix, row);
  if (rf.af) sell_row_Bt_impl<T, D, NRB, G, 2>(ix, rf, vals, p, sub, acc);
  else if (rf.pk) sell_row_Bt_impl<T, D, NRB, G, 1>(ix, rf, vals, p, sub, acc);
  else sell_row_Bt_impl<T, D, NRB, G, 0>(ix, rf, vals, p, sub, acc);
}

#define GRID_STRIDE_ROWS(row, nrows)                                                      \
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < (nrows);      \
       row += (int64_t)gridDim.x * blockDim.x)

// XCD-aware row partition for kernels that gather: workgroups are dealt
// round-robin over the 8 XCDs (each with its own L2), so workgroup b works on
// eighth (b % 8) of the rows -- one z-slab of the internal ordering, whose
// x-gathers then stay in one L2.  Rows of an eighth are strided over its
// workgroups.  G lanes per row: thread t of the eighth serves row t / G as
// lane `sub` = t mod G of its group (G divides the block size).
// PERM (the index's slice schedule, may be null): the t-th 64-row slice of an
// eighth in launch order is slice PERM[t], a permutation inside the eighth
// (SellIdx::rperm); a wavefront's rows lie in one slice, so the lookup is a
// uniform load.
#define XCD_ROWS_G(row, sub, nrows, G, PERM)                                                \
  const int64_t xg_ = (gridDim.x % 8 == 0) ? gridDim.x / 8 : gridDim.x;                   \
  const int64_t xx_ = (gridDim.x % 8 == 0) ? blockIdx.x % 8 : 0;                          \
  const int64_t xi_ = (gridDim.x % 8 == 0) ? blockIdx.x / 8 : blockIdx.x;                 \
  const int64_t xn_ = (gridDim.x % 8 == 0) ? ((((nrows) + 7) / 8 + 63) / 64) * 64 : (nrows); \
  const int64_t xb_ = xx_ * xn_;                                                          \
  const int64_t xe_ = xb_ + xn_ < (nrows) ? xb_ + xn_ : (nrows);                          \
  const int sub = (int)(threadIdx.x % (G));                                               \
  const int32_t* const xp_ = (PERM);                                                      \
  for (int64_t xr_ = xb_ + (xi_ * blockDim.x + threadIdx.x) / (G); xr_ < xe_; xr_ += xg_ * blockDim.x / (G)) \
    if (const int64_t row = xp_ ? ((int64_t)xp_[__builtin_amdgcn_readfirstlane((int)(xr_ >> 6))] << 6) + (xr_ & 63) : xr_; true)

#define XCD_ROWS(row, nrows, PERM) XCD_ROWS_G(row, sub_unused_ [[maybe_unused]], nrows, 1, PERM)

// Row-group mapping without the XCD partition (streaming kernels).
#define GRID_STRIDE_ROWS_G(row, sub, nrows, G)                                             \
  const int sub = (int)(threadIdx.x % (G));                                               \
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / (G); row < (nrows); \
       row += (int64_t)gridDim.x * blockDim.x / (G))

// Per-lane partial sums of components sub W/G .. into a full W-slot array
// (the other slots 0), for the block reduction.
template <int W, int G>
__device__ __forceinline__ void expand_parts(const double (&pg)[W / G], int sub, double (&pf)[W]) {
  constexpr int WG = W / G;
#pragma unroll
  for (int w = 0; w < W; ++w) pf[w] = (w / WG == sub) ? pg[w % WG] : 0.0;
}

// ----------------------------------------------------------- SpMV kernels

// y = a * (S x) + b * yin   (yin may alias y; ignored when b == 0)
// IL: ix and vals are the interleaved copies.
template <typename T, int W, int G, typename TM = T, bool IL = false>
__global__ __launch_bounds__(kBlock) void k_spmv(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                 const T* __restrict__ x, T* y, T a, const T* yin, T b) {
  constexpr int WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    if constexpr (IL) sell_row_il<T, W, G, TM>(ix, vals, x, row, sub, acc);
    else sell_row<T, W, G, TM, (W / G == 1 ? 16 : W / G <= 2 ? 8 : 4)>(ix, vals, x, row, sub, acc);
    const int64_t o = row * W + sub * WG;
    // yin may alias y: every load of the row is issued before its stores
    T yi[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) yi[w] = b != T(0) ? yin[o + w] : T(0);
#pragma unroll
    for (int w = 0; w < WG; ++w) y[o + w] = fma(b, yi[w], a * acc[w]);
  }
}

// ------------------------------------------------ entry-split SELL rows
//
// Operators with few but long rows (the coarse levels of the pressure
// multigrid: a two-ring stencil of some 60-130 entries on a few thousand
// rows) leave too few wavefronts in flight when one lane walks a whole row,
// and each lane then waits on a long chain of dependent gathers.  Here E
// lanes share a row (E in {2, 4, 8, 16}): lane `sub` of the group takes the
// slots sub, sub + E, sub + 2E, ... and accumulates every component of
// them; a butterfly of lane exchanges then leaves the row sums in every lane
// of the group (each exchange adds the same two values in both lanes, so all
// E lanes hold the same bits).  A wavefront holds 64 / E consecutive rows
// starting at a multiple of 64 / E, so they share one slice.
template <typename T, int W, int E, typename TM, int F, bool DS, int U>
__device__ __forceinline__ void sell_row_es_impl(const SellIdx& ix, const SliceRef& r, const TM* __restrict__ vals,
                                                 const T* __restrict__ x, const T* __restrict__ ds, int sub,
                                                 T (&acc)[W]) {
  auto group = [&](auto Uc, int j) {
    constexpr int UU = decltype(Uc)::value;
    int32_t c[UU];
    T v[UU];
#pragma unroll
    for (int u = 0; u < UU; ++u) {
      c[u] = sell_col_f<F>(ix, r, j + E * u);
      v[u] = (T)__builtin_nontemporal_load(vals + r.beg + 64 * (j + E * u));
    }
    if constexpr (DS) {
#pragma unroll
      for (int u = 0; u < UU; ++u) v[u] *= ds[c[u]];
    }
    T xv[UU][W];
#pragma unroll
    for (int u = 0; u < UU; ++u)
#pragma unroll
      for (int w = 0; w < W; ++w) xv[u][w] = x[(int64_t)c[u] * W + w];
#pragma unroll
    for (int u = 0; u < UU; ++u)
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] = fma(v[u], xv[u][w], acc[w]);
  };
  int j = sub;
  for (; j + E * (U - 1) < r.width; j += E * U) group(std::integral_constant<int, U>{}, j);
  if constexpr (U > 2)
    for (; j + E < r.width; j += 2 * E) group(std::integral_constant<int, 2>{}, j);
  for (; j < r.width; j += E) group(std::integral_constant<int, 1>{}, j);
}

// acc = sum over the row's entries of v_j x[c_j][0..W) (v_j ds[c_j] when ds
// is given), in every lane of the row group.
template <typename T, int W, int E, typename TM>
__device__ __forceinline__ void sell_row_es(const SellIdx& ix, const TM* __restrict__ vals, const T* __restrict__ x,
                                            int64_t row, int sub, T (&acc)[W], const T* __restrict__ ds = nullptr) {
  constexpr int U = W <= 2 ? 8 : 4;
  const SliceRef r = slice_ref(ix, row);
  if (ds) {
    if (r.af) sell_row_es_impl<T, W, E, TM, 2, true, U>(ix, r, vals, x, ds, sub, acc);
    else if (r.pk) sell_row_es_impl<T, W, E, TM, 1, true, U>(ix, r, vals, x, ds, sub, acc);
    else sell_row_es_impl<T, W, E, TM, 0, true, U>(ix, r, vals, x, ds, sub, acc);
  } else {
    if (r.af) sell_row_es_impl<T, W, E, TM, 2, false, U>(ix, r, vals, x, ds, sub, acc);
    else if (r.pk) sell_row_es_impl<T, W, E, TM, 1, false, U>(ix, r, vals, x, ds, sub, acc);
    else sell_row_es_impl<T, W, E, TM, 0, false, U>(ix, r, vals, x, ds, sub, acc);
  }
#pragma unroll
  for (int o = E / 2; o >= 1; o /= 2)
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] += __shfl_xor(acc[w], o);
}

// Entry-split forms of k_spmv, k_cheb_first (column scaling gathered) and
// k_cheb_step (no fused dot): the same arithmetic per row; lane `sub` of a
// row group stores the components w with w mod E == sub.
template <typename T, int W, int E, typename TM = T>
__global__ __launch_bounds__(kBlock) void k_spmv_es(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                    const T* __restrict__ x, T* y, T a, const T* yin, T b) {
  XCD_ROWS_G(row, sub, nrows, E, ix.rperm) {
    T acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    sell_row_es<T, W, E, TM>(ix, vals, x, row, sub, acc);
    const int64_t o = row * W;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (w % E != sub) continue;
      const T yi = b != T(0) ? yin[o + w] : T(0);
      y[o + w] = fma(b, yi, a * acc[w]);
    }
  }
}

template <typename T, int W, int ACC, int E, typename TM = T>
__global__ __launch_bounds__(kBlock) void k_cheb_first_es(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                          T ms, const T* __restrict__ r, const T* __restrict__ dinv,
                                                          T theta_inv, T* __restrict__ d1, T* __restrict__ res,
                                                          T* __restrict__ z, T c1, T c2) {
  XCD_ROWS_G(row, sub, nrows, E, ix.rperm) {
    T acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    sell_row_es<T, W, E, TM>(ix, vals, r, row, sub, acc, dinv);
    const T di = dinv[row];
    const int64_t o = row * W;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (w % E != sub) continue;
      const int64_t i = o + w;
      const T d0 = theta_inv * di * r[i];
      const T rs = r[i] - theta_inv * (ms * acc[w]);
      res[i] = rs;
      const T dnv = fma(c1, d0, c2 * di * rs);
      d1[i] = dnv;
      z[i] = ACC ? z[i] + (d0 + dnv) : d0 + dnv;
    }
  }
}

template <typename T, int W, int E, typename TM = T>
__global__ __launch_bounds__(kBlock) void k_cheb_step_es(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                         T ms, const T* __restrict__ d, T* __restrict__ dn,
                                                         const T* res_in, T* res_out, T* __restrict__ z,
                                                         const T* __restrict__ dinv, T c1, T c2) {
  XCD_ROWS_G(row, sub, nrows, E, ix.rperm) {
    T acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    sell_row_es<T, W, E, TM>(ix, vals, d, row, sub, acc);
    const T di = c2 * dinv[row];
    const int64_t o = row * W;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (w % E != sub) continue;
      // res_in may alias res_out: this lane alone reads and then writes o + w
      const T rs = res_in[o + w] - ms * acc[w];
      res_out[o + w] = rs;
      const T dnew = fma(c1, d[o + w], di * rs);
      dn[o + w] = dnew;
      z[o + w] += dnew;
    }
  }
}

// CG direction step with the product folded in:
//   q = S z (+ extra) + beta q,  p = z + beta p,  sigma = p . q  -> alpha
template <typename T, int W, int G>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(int64_t nrows, SellIdx ix,
                                                    const T* __restrict__ vals, const T* __restrict__ z,
                                                    const T* __restrict__ extra, T* __restrict__ q,
                                                    T* __restrict__ p, Scalars* sc, int cps, int nsys, double* partials) {
  constexpr int WG = W / G;
  const int sub0 = (int)(threadIdx.x % G);
  T beta[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) beta[w] = (T)sc->beta[(sub0 * WG + w) / cps];
  double part[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) part[w] = 0;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    if (ix.sp) sell_row<T, W, G>(ix, vals, z, row, sub, acc);
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = row * W + sub * WG + w;
      T a = acc[w];
      if (extra) a += extra[i];
      const T qn = fma(beta[w], q[i], a);
      const T pn = fma(beta[w], p[i], z[i]);
      q[i] = qn;
      p[i] = pn;
      part[w] += (double)pn * (double)qn;
    }
  }
  double pf[W];
  expand_parts<W, G>(part, sub0, pf);
  grid_reduce<W>(pf, partials);
}

// PREC: 0 = Chebyshev prologue (d0 = dinv r / theta, z = d0), 1 = Jacobi
// (z = dinv r, rho = r . z), 2 = none (the preconditioner runs separately).
// Always: x += alpha p, r -= alpha q, rr = r . r.
template <typename T, int W, int PREC, int G>
__global__ __launch_bounds__(kBlock) void k_cg_update(int64_t nrows, T* __restrict__ x, T* __restrict__ r,
                                                      const T* __restrict__ p, const T* __restrict__ q,
                                                      const T* __restrict__ dinv, T theta_inv, T* __restrict__ d0,
                                                      T* __restrict__ z, Scalars* sc, int cps, int nsys, double* partials) {
  constexpr int WG = W / G;
  const int sub0 = (int)(threadIdx.x % G);
  T alpha[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) alpha[w] = (T)sc->alpha[(sub0 * WG + w) / cps];
  double prr[WG], prz[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) prr[w] = prz[w] = 0;
  GRID_STRIDE_ROWS_G(row, sub, nrows, G) {
    const T di = PREC == 2 ? T(0) : dinv[row];  // one inverse diagonal per node
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = row * W + sub * WG + w;
      x[i] = fma(alpha[w], p[i], x[i]);
      const T rn = fma(-alpha[w], q[i], r[i]);
      r[i] = rn;
      prr[w] += (double)rn * (double)rn;
      if (PREC == 0) {
        const T dd = rn * di * theta_inv;
        d0[i] = dd;
        z[i] = dd;
      } else if (PREC == 1) {
        const T zz = rn * di;
        z[i] = zz;
        prz[w] += (double)rn * (double)zz;
      }
    }
  }
  constexpr int NS = PREC == 1 ? 2 * W : W;
  double pf[NS], t[W];
  expand_parts<W, G>(prr, sub0, t);
#pragma unroll
  for (int w = 0; w < W; ++w) pf[w] = t[w];
  if constexpr (PREC == 1) {
    expand_parts<W, G>(prz, sub0, t);
#pragma unroll
    for (int w = 0; w < W; ++w) pf[W + w] = t[w];
  }
  grid_reduce<NS>(pf, partials);
}

// Chebyshev prologue on its own: d0 = dinv r / theta, z = d0.
template <typename T, int W, int G>
__global__ __launch_bounds__(kBlock) void k_cheb_init(int64_t nrows, const T* __restrict__ r,
                                                      const T* __restrict__ dinv, T theta_inv, T* __restrict__ d0,
                                                      T* __restrict__ z) {
  constexpr int WG = W / G;
  GRID_STRIDE_ROWS_G(row, sub, nrows, G) {
    const T di = dinv[row] * theta_inv;
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = row * W + sub * WG + w;
      const T dd = r[i] * di;
      d0[i] = dd;
      z[i] = dd;
    }
  }
}

// One Chebyshev step (Saad, Iterative Methods, Alg. 12.1, three-term form):
//   res = res_in - S d ;  dn = c1 d + c2 dinv res ;  z += dn
// DOT: also rho = rvec . z -> beta (CG preconditioner use), first => beta = 0.
template <typename T, int W, int DOT, int G, typename TM = T>
__global__ __launch_bounds__(kBlock) void k_cheb_step(int64_t nrows, SellIdx ix,
                                                      const TM* __restrict__ vals, T ms, const T* __restrict__ d,
                                                      T* __restrict__ dn, const T* res_in, T* res_out,
                                                      T* __restrict__ z, const T* __restrict__ dinv, T c1, T c2,
                                                      const T* __restrict__ rvec, Scalars* sc, int cps, int nsys,
                                                      int first, double* partials) {
  constexpr int WG = W / G;
  double part[WG];
#pragma unroll
  for (int w = 0; w < WG; ++w) part[w] = 0;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    sell_row<T, W, G, TM, (W / G == 1 ? 16 : W / G <= 2 ? 8 : 4)>(ix, vals, d, row, sub, acc);
    const T di = c2 * dinv[row];
    const int64_t o = row * W + sub * WG;
    // res_in may alias res_out: load the whole row before any store
    T ri[WG], dd[WG], zz[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      ri[w] = res_in[o + w];
      dd[w] = d[o + w];
      zz[w] = z[o + w];
    }
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const T rs = ri[w] - ms * acc[w];
      res_out[o + w] = rs;
      const T dnew = fma(c1, dd[w], di * rs);
      dn[o + w] = dnew;
      const T zn = zz[w] + dnew;
      z[o + w] = zn;
      if (DOT) part[w] += (double)rvec[o + w] * (double)zn;
    }
  }
  if (DOT) {
    double pf[W];
    expand_parts<W, G>(part, (int)(threadIdx.x % G), pf);
    grid_reduce<W>(pf, partials);
  }
}

// First Chebyshev step with the prologue folded in: d0 = theta_inv dinv r is
// formed on the fly at every gathered column, so no separate pass is needed:
//   res = r - S d0 ;  d1 = c1 d0 + c2 dinv res ;  z = d0 + d1
// ACC: z += d0 + d1 (z holds a previous approximation) instead of z = d0 + d1
// SC: vals already hold S_ij dinv_j (no gather of dinv at the columns).
template <typename T, int W, int ACC, int G, int SC, typename TM = T>
__global__ __launch_bounds__(kBlock) void k_cheb_first(int64_t nrows, SellIdx ix, const TM* __restrict__ vals, T ms,
                                                       const T* __restrict__ r, const T* __restrict__ dinv, T theta_inv,
                                                       T* __restrict__ d1, T* __restrict__ res, T* __restrict__ z,
                                                       T c1, T c2) {
  constexpr int WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    sell_row<T, W, G, TM, (W / G == 1 ? 16 : W / G <= 2 ? 8 : 4)>(ix, vals, r, row, sub, acc, SC ? nullptr : dinv);
    const T di = dinv[row];
    const int64_t o = row * W + sub * WG;
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = o + w;
      const T d0 = theta_inv * di * r[i];
      const T rs = r[i] - theta_inv * (ms * acc[w]);
      res[i] = rs;
      const T dnv = fma(c1, d0, c2 * di * rs);
      d1[i] = dnv;
      z[i] = ACC ? z[i] + (d0 + dnv) : d0 + dnv;
    }
  }
}

// Chebyshev steps on the column-scaled operator S D^{-1} held as TM (the
// half-precision copy of the velocity block), in the variable q = D d:
//   S d = (S D^{-1}) q,  and  dn = c1 d + c2 dinv res  becomes  qn = c1 q + c2 res,
// with z += dinv qn.  The iterates z and res are those of k_cheb_first /
// k_cheb_step up to rounding; only the stored direction is rescaled.
//
// First step (q0 = theta_inv r):
//   res = r - (S D^{-1}) q0 ;  q1 = c1 q0 + c2 res ;  z = dinv (q0 + q1)  (ACC: z +=)
template <typename T, typename TM, int W, int ACC, int G, int U = 4>
__global__ __launch_bounds__(kBlock) void k_cheb_first_q(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                         const T* __restrict__ r, const T* __restrict__ dinv,
                                                         T theta_inv, T* __restrict__ q1, T* __restrict__ res,
                                                         T* __restrict__ z, T c1, T c2) {
  constexpr int WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    sell_row<T, W, G, TM, U>(ix, vals, r, row, sub, acc);
    const T di = dinv[row];
    const int64_t o = row * W + sub * WG;
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = o + w;
      const T q0 = theta_inv * r[i];
      const T rs = r[i] - theta_inv * acc[w];
      res[i] = rs;
      const T qn = fma(c1, q0, c2 * rs);
      q1[i] = qn;
      z[i] = ACC ? fma(di, q0 + qn, z[i]) : di * (q0 + qn);
    }
  }
}

// Later steps:  res = res_in - (S D^{-1}) q ;  qn = c1 q + c2 res ;  z += dinv qn
// U: entries per unrolled group (8 keeps twice the loads of the 2-byte
// value and 1-byte index streams in flight; 4% faster than 4 at W = 3).
template <typename T, typename TM, int W, int G, int U = 4>
__global__ __launch_bounds__(kBlock) void k_cheb_step_q(int64_t nrows, SellIdx ix,
                                                        const TM* __restrict__ vals, const T* __restrict__ q,
                                                        T* __restrict__ qn, const T* res_in, T* res_out,
                                                        T* __restrict__ z, const T* __restrict__ dinv, T c1, T c2) {
  constexpr int WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    const int64_t o = row * W + sub * WG;
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    sell_row<T, W, G, TM, U>(ix, vals, q, row, sub, acc);
    // res_in may alias res_out: load the whole row before any store
    T ri[WG], qq[WG], zz[WG];
    const T di = dinv[row];
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      ri[w] = res_in[o + w];
      qq[w] = q[o + w];
      zz[w] = z[o + w];
    }
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const T rs = ri[w] - acc[w];
      res_out[o + w] = rs;
      const T qnew = fma(c1, qq[w], c2 * rs);
      qn[o + w] = qnew;
      z[o + w] = fma(di, qnew, zz[w]);
    }
  }
}

// ------------------------------------------ bfloat16 Chebyshev directions
// The velocity Chebyshev polynomial may keep its direction q in bfloat16
// (FP32 exponent range, 8-bit mantissa): it only shapes the preconditioner,
// and the residual and z are updated with the rounded q, so the recurrence
// stays consistent.  Rows of W values are stored WP = (W == 3 ? 4 : W) wide
// (one aligned 8-byte load per gathered node at W = 3; the pad is 0).
__device__ __forceinline__ uint16_t bf16_of(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float f_of_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

template <int W>
__host__ __device__ constexpr int bf_width() { return W == 3 ? 4 : W; }

// out[0..WG) = row values at component offset `off` of node c (WP per node)
template <int WP, int WG>
__device__ __forceinline__ void load_bf(const uint16_t* __restrict__ xq, int64_t c, int off, float (&out)[WG]) {
  if constexpr (WP == 4 && WG >= 3) {
    const uint2 u = *reinterpret_cast<const uint2*>(xq + c * 4);
    out[0] = __uint_as_float(u.x << 16);
    out[1] = __uint_as_float(u.x & 0xFFFF0000u);
    out[2] = __uint_as_float(u.y << 16);
    if constexpr (WG == 4) out[3] = __uint_as_float(u.y & 0xFFFF0000u);
  } else if constexpr (WG % 2 == 0 && WP % 2 == 0) {
    // pairs of values as 32-bit words (c WP and off are even: 4-byte aligned)
    const uint32_t* p = reinterpret_cast<const uint32_t*>(xq + c * WP + off);
#pragma unroll
    for (int k = 0; k < WG / 2; ++k) {
      const uint32_t u = p[k];
      out[2 * k] = __uint_as_float(u << 16);
      out[2 * k + 1] = __uint_as_float(u & 0xFFFF0000u);
    }
  } else {
#pragma unroll
    for (int w = 0; w < WG; ++w) out[w] = f_of_bf16(xq[c * WP + off + w]);
  }
}

// Packed form of a gathered row: 32-bit words holding two bfloat16 values
// each, unpacked only where the products use them, so that an unrolled group
// keeps half as many registers in flight as with the values widened to FP32.
template <int WP, int WG>
struct BfRaw {
  static constexpr bool kOn = (WP == 4 && WG >= 3) || (WG % 2 == 0 && WP % 2 == 0);
  static constexpr int kWords = WP == 4 && WG >= 3 ? 2 : WG / 2;
};

template <int WP, int WG>
__device__ __forceinline__ void load_bf_raw(const uint16_t* __restrict__ xq, int64_t c, int off,
                                            uint32_t (&raw)[BfRaw<WP, WG>::kWords]) {
  if constexpr (WP == 4 && WG >= 3) {
    const uint2 u = *reinterpret_cast<const uint2*>(xq + c * 4);
    raw[0] = u.x;
    raw[1] = u.y;
  } else {
    const uint32_t* p = reinterpret_cast<const uint32_t*>(xq + c * WP + off);
#pragma unroll
    for (int k = 0; k < WG / 2; ++k) raw[k] = p[k];
  }
}

// component w of a packed row (the low half of a word is the even component)
__device__ __forceinline__ float bf_word(uint32_t u, int hi) {
  return __uint_as_float(hi ? (u & 0xFFFF0000u) : (u << 16));
}

template <int W, int G, typename TM, int F, int U>
__device__ __forceinline__ void sell_row_bq_impl(const SellIdx& ix, const SliceRef& r, const TM* __restrict__ vals,
                                                 const uint16_t* __restrict__ xq, int off, float (&acc)[W / G]) {
  constexpr int WG = W / G, WP = bf_width<W>();
  using Raw = BfRaw<WP, WG>;
  auto group = [&](auto Uc, int j) {
    constexpr int UU = decltype(Uc)::value;
    int32_t c[UU];
    float v[UU];
#pragma unroll
    for (int u = 0; u < UU; ++u) {
      c[u] = sell_col_f<F>(ix, r, j + u);
      v[u] = (float)__builtin_nontemporal_load(vals + r.beg + 64 * (j + u));
    }
    if constexpr (Raw::kOn) {
      uint32_t xr[UU][Raw::kWords];
#pragma unroll
      for (int u = 0; u < UU; ++u) load_bf_raw<WP, WG>(xq, c[u], off, xr[u]);
#pragma unroll
      for (int u = 0; u < UU; ++u)
#pragma unroll
        for (int w = 0; w < WG; ++w) acc[w] = fma(v[u], bf_word(xr[u][w / 2], w & 1), acc[w]);
    } else {
      float xv[UU][WG];
#pragma unroll
      for (int u = 0; u < UU; ++u) load_bf<WP, WG>(xq, c[u], off, xv[u]);
#pragma unroll
      for (int u = 0; u < UU; ++u)
#pragma unroll
        for (int w = 0; w < WG; ++w) acc[w] = fma(v[u], xv[u][w], acc[w]);
    }
  };
  int j = 0;
  for (; j + U <= r.width; j += U) group(std::integral_constant<int, U>{}, j);
  if constexpr (U > 4)
    for (; j + 4 <= r.width; j += 4) group(std::integral_constant<int, 4>{}, j);
  for (; j < r.width; ++j) group(std::integral_constant<int, 1>{}, j);
}

// The bfloat16-direction row over the interleaved half-precision copies
// (the layout of sell_row_il_impl, eight slots per group).
template <int W, int G, int F>
__device__ __forceinline__ void sell_row_bq_il_impl(const SellIdx& ix, const SliceRef& r,
                                                  const _Float16* __restrict__ vals,
                                                  const uint16_t* __restrict__ xq, int off, float (&acc)[W / G]) {
  constexpr int WG = W / G, WP = bf_width<W>(), IW = il_width<_Float16>();
  using Raw = BfRaw<WP, WG>;
  static_assert(Raw::kOn, "interleaved rows take the packed bfloat16 gathers");
  const int64_t s0 = r.eb << 6;
  const int lr = static_cast<int>(r.beg - s0);
  const int gi = r.width / IW;
  auto entry = [&](int g) { return s0 + 64 * IW * (int64_t)g + IW * lr; };
  // H groups at a time: values and offsets first, then all their gathers
  auto groups = [&](auto Hc, int g) {
    constexpr int H = decltype(Hc)::value;
    int32_t c[H][IW];
    float v[H][IW];
#pragma unroll
    for (int h = 0; h < H; ++h) {
      load_vals<IW, _Float16, float>(vals, entry(g + h), v[h]);
      load_cols<IW, F>(ix, r, g + h, entry(g + h), c[h]);
    }
    uint32_t xr[H][IW][Raw::kWords];
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int k = 0; k < IW; ++k) load_bf_raw<WP, WG>(xq, c[h][k], off, xr[h][k]);
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int k = 0; k < IW; ++k)
#pragma unroll
        for (int w = 0; w < WG; ++w) acc[w] = fma(v[h][k], bf_word(xr[h][k][w / 2], w & 1), acc[w]);
  };
  // narrow lanes keep two groups (16 entries) in flight, wide ones one
  constexpr int HG = WG <= 4 ? 2 : 1;
  int g = 0;
  if constexpr (F == 2 && WP == 4 && WG >= 3) {
    // 8-byte rows: the leading pair sub-groups (four slots 4p .. 4p+3 of
    // which slots 4p, 4p+1 and 4p+2, 4p+3 gather adjacent nodes in every
    // lane; r.pg of them) take one 16-byte gather per pair.  NP: pairs of
    // the group taken that way (4, or 2 for a group half made of pairs).
    auto pairs = [&](auto Hc, auto NPc, int g0) {
      constexpr int H = decltype(Hc)::value, NP = decltype(NPc)::value;
      int32_t c[H][IW];
      float v[H][IW];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        load_vals<IW, _Float16, float>(vals, entry(g0 + h), v[h]);
#pragma unroll
        for (int k = 0; k < IW; ++k)
          if (k < 2 * NP ? k % 2 == 0 : true) c[h][k] = affine_col(ix, r, r.eb + IW * (g0 + h) + k);
      }
      u32x4a8_t u[H][NP];
      uint32_t xr[H][IW][Raw::kWords];
#pragma unroll
      for (int h = 0; h < H; ++h) {
#pragma unroll
        for (int p = 0; p < NP; ++p) u[h][p] = *reinterpret_cast<const u32x4a8_t*>(xq + (int64_t)c[h][2 * p] * 4);
#pragma unroll
        for (int k = 2 * NP; k < IW; ++k) load_bf_raw<WP, WG>(xq, c[h][k], off, xr[h][k]);
      }
#pragma unroll
      for (int h = 0; h < H; ++h) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          xr[h][2 * p][0] = u[h][p].x;
          xr[h][2 * p][1] = u[h][p].y;
          xr[h][2 * p + 1][0] = u[h][p].z;
          xr[h][2 * p + 1][1] = u[h][p].w;
        }
#pragma unroll
        for (int k = 0; k < IW; ++k)
#pragma unroll
          for (int w = 0; w < WG; ++w) acc[w] = fma(v[h][k], bf_word(xr[h][k][w / 2], w & 1), acc[w]);
      }
    };
    const int gp = r.pg / 2;  // groups made of four pairs
    for (; g + 2 <= gp; g += 2) pairs(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{}, g);
    for (; g < gp; ++g) pairs(std::integral_constant<int, 1>{}, std::integral_constant<int, 4>{}, g);
    if ((r.pg & 1) && g < gi) pairs(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{}, g++);
  }
  for (; g + HG <= gi; g += HG) groups(std::integral_constant<int, HG>{}, g);
  if (g < gi) groups(std::integral_constant<int, 1>{}, g);
  // the remaining width mod IW slots, slot-major
  for (int j = IW * gi; j < r.width; ++j) {
    const int32_t c = sell_col_f<F>(ix, r, j);
    const float v = (float)__builtin_nontemporal_load(vals + r.beg + 64 * j);
    uint32_t xr[Raw::kWords];
    load_bf_raw<WP, WG>(xq, c, off, xr);
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = fma(v, bf_word(xr[w / 2], w & 1), acc[w]);
  }
}

// Permute one scalar array of a sliced-ELL layout into the interleaved order
// above with IW slots per group (one workgroup of 64 threads per slice).
template <typename E, int IW>
__global__ __launch_bounds__(64) void k_interleave(int64_t nslices, const int64_t* __restrict__ sp,
                                                   const E* __restrict__ src, E* __restrict__ dst) {
  const int64_t s = blockIdx.x;
  if (s >= nslices) return;
  const int64_t s0 = sp[s];
  const int w = static_cast<int>((sp[s + 1] - s0) >> 6);
  const int lr = threadIdx.x, gi = w / IW;
  for (int j = 0; j < w; ++j) {
    const int64_t from = s0 + 64 * (int64_t)j + lr;
    const int64_t to = j < IW * gi ? s0 + 64 * IW * (int64_t)(j / IW) + IW * lr + (j % IW) : from;
    dst[to] = src[from];
  }
}

// The closing step of a deferred Chebyshev sum (the iterate is not carried
// through the steps): z = dinv (theta_inv r + q_1 + ... + q_n + q_last),
// with the directions q_k = D d_k kept in bfloat16.
constexpr int kQSumMax = 14;
struct QSum {
  const float* r;
  float theta_inv;
  int n;
  const uint16_t* q[kQSumMax];
};

// First step with a bfloat16 direction out:  q0 = theta_inv r (not stored),
// res = r - (S D^{-1}) q0, q1 = bf16(c1 q0 + c2 res), z (+)= dinv (q0 + q1);
// ACC = 2 leaves z to the closing step (no z, no dinv).
// IL: ix and vals are the interleaved copies.
template <typename TM, int W, int ACC, int G, int U = 8, bool IL = false>
__global__ __launch_bounds__(kBlock) void k_cheb_first_qb(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                          const float* __restrict__ r, const float* __restrict__ dinv,
                                                          float theta_inv, uint16_t* __restrict__ q1,
                                                          float* __restrict__ res, float* __restrict__ z, float c1,
                                                          float c2) {
  constexpr int WG = W / G, WP = bf_width<W>();
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    float acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    if constexpr (IL) sell_row_il<float, W, G, TM>(ix, vals, r, row, sub, acc);
    else sell_row<float, W, G, TM, (W / G >= 8 ? 4 : U)>(ix, vals, r, row, sub, acc);
    const float di = ACC == 2 ? 0.f : dinv[row];
    const int64_t o = row * W + sub * WG, oq = row * WP + sub * WG;
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const int64_t i = o + w;
      const float q0 = theta_inv * r[i];
      const float rs = r[i] - theta_inv * acc[w];
      res[i] = rs;
      const uint16_t qb = bf16_of(fma(c1, q0, c2 * rs));
      q1[oq + w] = qb;
      const float qn = f_of_bf16(qb);
      if constexpr (ACC == 1) z[i] = fma(di, q0 + qn, z[i]);
      else if constexpr (ACC == 0) z[i] = di * (q0 + qn);
    }
    if constexpr (WP != W) {
      if (sub == G - 1) q1[row * WP + W] = 0;
    }
  }
}

// Later steps:  res = res_in - (S D^{-1}) q ;  qn = bf16(c1 q + c2 res) ;  z += dinv qn
// ZM = 1: the deferred form -- no z (nor dinv); ZM = 2: the closing step --
// neither res nor qn is stored, z = dinv (fin.theta_inv fin.r + fin.q[0] +
// ... + fin.q[n-1] + qn).
// IL: ix.cdel / ix.cols and vals are the interleaved copies.
template <typename TM, int W, int G, int U = 8, bool IL = false, int ZM = 0>
__global__ __launch_bounds__(kBlock) void k_cheb_step_qb(int64_t nrows, SellIdx ix, const TM* __restrict__ vals,
                                                         const uint16_t* __restrict__ q, uint16_t* __restrict__ qn,
                                                         const float* res_in, float* res_out, float* __restrict__ z,
                                                         const float* __restrict__ dinv, float c1, float c2,
                                                         QSum fin) {
  constexpr int WG = W / G, WP = bf_width<W>();
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    const int64_t o = row * W + sub * WG;
    float acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    {
      const SliceRef rf = slice_ref(ix, row);
      // wide lanes (8 or more components) take four entries per group: with
      // eight, the gathered words alone hold most of the registers
      constexpr int UB = WG >= 8 ? 4 : U;
      if constexpr (IL) {
        if (rf.af) sell_row_bq_il_impl<W, G, 2>(ix, rf, vals, q, sub * WG, acc);
        else if (rf.pk) sell_row_bq_il_impl<W, G, 1>(ix, rf, vals, q, sub * WG, acc);
        else sell_row_bq_il_impl<W, G, 0>(ix, rf, vals, q, sub * WG, acc);
      } else {
        if (rf.af) sell_row_bq_impl<W, G, TM, 2, UB>(ix, rf, vals, q, sub * WG, acc);
        else if (rf.pk) sell_row_bq_impl<W, G, TM, 1, UB>(ix, rf, vals, q, sub * WG, acc);
        else sell_row_bq_impl<W, G, TM, 0, UB>(ix, rf, vals, q, sub * WG, acc);
      }
    }
    // res_in may alias res_out: load the whole row before any store
    float ri[WG], qq[WG], zz[WG];
    const float di = ZM == 1 ? 0.f : dinv[row];
    load_bf<WP, WG>(q, row, sub * WG, qq);
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      ri[w] = res_in[o + w];
      if constexpr (ZM == 0) zz[w] = z[o + w];
    }
    if constexpr (ZM == 2) {
      // the earlier directions, summed in step order after theta_inv r
#pragma unroll
      for (int w = 0; w < WG; ++w) zz[w] = fin.theta_inv * fin.r[o + w];
      for (int k = 0; k < fin.n; ++k) {
        float t[WG];
        load_bf<WP, WG>(fin.q[k], row, sub * WG, t);
#pragma unroll
        for (int w = 0; w < WG; ++w) zz[w] += t[w];
      }
    }
    const int64_t oq = row * WP + sub * WG;
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      const float rs = ri[w] - acc[w];
      if constexpr (ZM != 2) res_out[o + w] = rs;
      const uint16_t qb = bf16_of(fma(c1, qq[w], c2 * rs));
      if constexpr (ZM != 2) qn[oq + w] = qb;
      if constexpr (ZM == 0) z[o + w] = fma(di, f_of_bf16(qb), zz[w]);
      else if constexpr (ZM == 2) z[o + w] = di * (zz[w] + f_of_bf16(qb));
    }
    if constexpr (WP != W && ZM != 2) {
      if (sub == G - 1) qn[row * WP + W] = 0;
    }
  }
}

// ------------------------------------------------------------- B and B^T

// p = a * (B u) + b * pin
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_B(int64_t nrows, SellIdx ix, const T* __restrict__ vals,
                                              const T* __restrict__ u, T* pout, T a, const T* pin, T b) {
  XCD_ROWS(row, nrows, ix.rperm) {
    T acc[NRB];
#pragma unroll
    for (int r = 0; r < NRB; ++r) acc[r] = 0;
    sell_row_B<T, D, NRB>(ix, vals, u, row, acc);
    T pi[NRB];  // pin may alias pout
#pragma unroll
    for (int r = 0; r < NRB; ++r) pi[r] = b != T(0) ? pin[row * NRB + r] : T(0);
#pragma unroll
    for (int r = 0; r < NRB; ++r) pout[row * NRB + r] = fma(b, pi[r], a * acc[r]);
  }
}

// u = a * scale .* (B^T p) + b * uin     (scale per node, may be null)
template <typename T, int D, int NRB, int G>
__global__ __launch_bounds__(kBlock) void k_Bt(int64_t nrows, SellIdx ix, const T* __restrict__ vals,
                                               const T* __restrict__ p, const T* __restrict__ scale, T* uout,
                                               T a, const T* uin, T b, T* __restrict__ btout) {
  constexpr int W = D * NRB, WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ix.rperm) {
    T acc[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = 0;
    sell_row_Bt<T, D, NRB, G>(ix, vals, p, row, sub, acc);
    const T sc = scale ? a * scale[row] : a;
    const int64_t o = row * W + sub * WG;
    T ui[WG];  // uin may alias uout
#pragma unroll
    for (int w = 0; w < WG; ++w) ui[w] = b != T(0) ? uin[o + w] : T(0);
#pragma unroll
    for (int w = 0; w < WG; ++w) uout[o + w] = fma(b, ui[w], sc * acc[w]);
    if (btout) {  // the scaled product alone, for reuse
#pragma unroll
      for (int w = 0; w < WG; ++w) btout[o + w] = sc * acc[w];
    }
  }
}

// Momentum rows of the coupled operator:
//   y = sgn * (A u - B^T p + extra) + yin   (sgn = -1 with yin = F gives the residual)
template <typename T, int D, int NRB, int G>
__global__ __launch_bounds__(kBlock) void k_momentum(int64_t nrows, SellIdx ixA, const T* __restrict__ A,
                                                     SellIdx ixT, const T* __restrict__ Bt,
                                                     const T* __restrict__ u, const T* __restrict__ p,
                                                     const T* __restrict__ extra, T* y, T sgn, const T* yin) {
  constexpr int W = D * NRB, WG = W / G;
  XCD_ROWS_G(row, sub, nrows, G, ixA.rperm) {
    T acc[WG], bt[WG];
#pragma unroll
    for (int w = 0; w < WG; ++w) acc[w] = bt[w] = 0;
    sell_row<T, W, G>(ixA, A, u, row, sub, acc);
    sell_row_Bt<T, D, NRB, G>(ixT, Bt, p, row, sub, bt);
    const int64_t o = row * W + sub * WG;
    T ex[WG], yi[WG];  // yin may alias y
#pragma unroll
    for (int w = 0; w < WG; ++w) {
      ex[w] = extra ? extra[o + w] : T(0);
      yi[w] = yin ? yin[o + w] : T(0);
    }
#pragma unroll
    for (int w = 0; w < WG; ++w) y[o + w] = fma(sgn, acc[w] - bt[w] + ex[w], yi[w]);
  }
}

// ---------------------------------------------- strain-form velocity block
// The velocity block alpha M + mu (L + D) couples the components: entry k of
// the sliced-ELL pattern carries a symmetric dim x dim block, stored as its
// P = dim (dim + 1) / 2 upper entries in plane-major groups of 64 entries
// (plane e of entry k at (k - k mod 64) P + 64 e + k mod 64), and
// y[row][r][a] += sum_b V[k][a][b] x[col][r][b] for every right-hand side.
template <int D>
__device__ __forceinline__ constexpr int sym_index(int a, int b) {
  // row-major position of (min, max) among the upper entries
  return a <= b ? a * D - a * (a - 1) / 2 + (b - a) : b * D - b * (b - 1) / 2 + (a - b);
}

template <typename T, int D, int NRB, int F>
__device__ __forceinline__ void sell_row_blk_impl(const SellIdx& ix, const SliceRef& rf, const T* __restrict__ vals,
                                                  const T* __restrict__ x, int64_t row, T (&acc)[D * NRB]) {
  constexpr int W = D * NRB, DD = D * (D + 1) / 2;
  const T* __restrict__ vrow = vals + (rf.beg - (row & 63)) * DD + (row & 63);
  constexpr int U = 2;
  int j = 0;
  for (; j + U <= rf.width; j += U) {
    int32_t c[U];
    T v[U][DD], xv[U][W];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      c[q] = sell_col_f<F>(ix, rf, j + q);
#pragma unroll
      for (int e = 0; e < DD; ++e) v[q][e] = __builtin_nontemporal_load(vrow + (int64_t)(j + q) * 64 * DD + 64 * e);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int w = 0; w < W; ++w) xv[q][w] = x[(int64_t)c[q] * W + w];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b)
            acc[r * D + a] = fma(v[q][sym_index<D>(a, b)], xv[q][r * D + b], acc[r * D + a]);
  }
  for (; j < rf.width; ++j) {
    const int32_t c = sell_col_f<F>(ix, rf, j);
    T v[DD];
#pragma unroll
    for (int e = 0; e < DD; ++e) v[e] = __builtin_nontemporal_load(vrow + (int64_t)j * 64 * DD + 64 * e);
    const T* xp = x + (int64_t)c * W;
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) acc[r * D + a] = fma(v[sym_index<D>(a, b)], xp[r * D + b], acc[r * D + a]);
  }
}

template <typename T, int D, int NRB>
__device__ __forceinline__ void sell_row_blk(const SellIdx& ix, const T* __restrict__ vals, const T* __restrict__ x,
                                             int64_t row, T (&acc)[D * NRB]) {
  const SliceRef rf = slice_ref(ix, row);
  if (rf.af) sell_row_blk_impl<T, D, NRB, 2>(ix, rf, vals, x, row, acc);
  else if (rf.pk) sell_row_blk_impl<T, D, NRB, 1>(ix, rf, vals, x, row, acc);
  else sell_row_blk_impl<T, D, NRB, 0>(ix, rf, vals, x, row, acc);
}

// y = a * (A x) + b * yin with the block operator (yin may alias y)
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_spmv_blk(int64_t nrows, SellIdx ix, const T* __restrict__ vals,
                                                     const T* __restrict__ x, T* y, T a, const T* yin, T b) {
  constexpr int W = D * NRB;
  XCD_ROWS(row, nrows, ix.rperm) {
    T acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    sell_row_blk<T, D, NRB>(ix, vals, x, row, acc);
    T yi[W];
#pragma unroll
    for (int w = 0; w < W; ++w) yi[w] = b != T(0) ? yin[row * W + w] : T(0);
#pragma unroll
    for (int w = 0; w < W; ++w) y[row * W + w] = fma(b, yi[w], a * acc[w]);
  }
}

// Momentum rows with the block operator: y = sgn (A u - B^T p + extra) + yin
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_momentum_blk(int64_t nrows, SellIdx ixA, const T* __restrict__ A,
                                                         SellIdx ixT, const T* __restrict__ Bt,
                                                         const T* __restrict__ u, const T* __restrict__ p,
                                                         const T* __restrict__ extra, T* y, T sgn, const T* yin) {
  constexpr int W = D * NRB;
  XCD_ROWS(row, nrows, ixA.rperm) {
    T acc[W], bt[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = bt[w] = 0;
    sell_row_blk<T, D, NRB>(ixA, A, u, row, acc);
    sell_row_Bt<T, D, NRB, 1>(ixT, Bt, p, row, 0, bt);
    T ex[W], yi[W];  // yin may alias y
#pragma unroll
    for (int w = 0; w < W; ++w) {
      ex[w] = extra ? extra[row * W + w] : T(0);
      yi[w] = yin ? yin[row * W + w] : T(0);
    }
#pragma unroll
    for (int w = 0; w < W; ++w) y[row * W + w] = fma(sgn, acc[w] - bt[w] + ex[w], yi[w]);
  }
}

// ------------------------------------------------------------ vector ops

// y = a x + b y
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpby(int64_t n, T a, const T* __restrict__ x, T b, T* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (b == T(0)) ? a * x[i] : fma(a, x[i], b * y[i]);
}

// y[i] = x[i] + s[slot] * v[i]  with per-system coefficients from device memory
template <typename T>
__global__ __launch_bounds__(kBlock) void k_axpy_sys(int64_t n, int W, int cps, const double* coef,
                                                     double scale, const T* __restrict__ v, T* y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int w = (int)(i % W);
    y[i] = fma((T)(scale * coef[w / cps]), v[i], y[i]);
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_cast(int64_t n, const Tin* __restrict__ x, Tout* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (Tout)x[i];
}

// out[w] = sum_rows x[row][w] * y[row][w]  (y null => x[row][w]^2); weight per
// row optional.  Result written to res[0..W) by the last block.
template <typename T, int W>
__global__ __launch_bounds__(kBlock) void k_dot(int64_t nrows, const T* __restrict__ x, const T* __restrict__ y,
                                                const double* __restrict__ rw, double* res, double* partials) {
  double part[W];
#pragma unroll
  for (int w = 0; w < W; ++w) part[w] = 0;
  GRID_STRIDE_ROWS(row, nrows) {
    const double wt = rw ? rw[row] : 1.0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const double a = x[row * W + w];
      const double b = y ? (double)y[row * W + w] : a;
      part[w] += wt * a * b;
    }
  }
  grid_reduce<W>(part, partials);
}

// x[row][r] -= shift[r]   (pressure mean removal; shift from device)
template <typename T, int NRB>
__global__ __launch_bounds__(kBlock) void k_shift(int64_t nrows, T* x, const double* __restrict__ sum,
                                                  double scale) {
  GRID_STRIDE_ROWS(row, nrows) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) x[row * NRB + r] -= (T)(sum[r] * scale);
  }
}

// dst[row][r] = src[row][r] - scale * (total of slot r over the block
// partials of a k_dot): every workgroup adds the partials itself, in the same
// fixed order, so all of them subtract the same bits and no separate
// finishing kernel runs.  dst may alias src.
template <typename T, int NRB>
__global__ __launch_bounds__(kBlock) void k_shift_p(int64_t nrows, const T* src, T* dst,
                                                    const double* __restrict__ partials, int nparts, double scale) {
  double a[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) a[r] = 0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) a[r] += partials[(size_t)b * NRB + r];
  }
  __shared__ double tot[NRB];
  block_sum<NRB>(a, tot);
  GRID_STRIDE_ROWS(row, nrows) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) dst[row * NRB + r] = src[row * NRB + r] - (T)(tot[r] * scale);
  }
}

// ------------------------------------------------------- layout transfers

// caller [nrb][D][n_p2] (double) -> internal [n_int][nrb][D] (T), interior only
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_vel_in(int64_t n_int, int64_t n_p2, const int32_t* __restrict__ int2nat,
                                                   const double* __restrict__ src, T* __restrict__ dst) {
  GRID_STRIDE_ROWS(row, n_int) {
    const int64_t nat = int2nat[row];
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int d = 0; d < D; ++d) dst[(row * NRB + r) * D + d] = (T)src[((int64_t)r * D + d) * n_p2 + nat];
  }
}

// internal -> caller (interior nodes); boundary nodes: ubc (or 0 if null) when
// bnd_fill != 0, untouched otherwise
template <typename T, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_vel_out(int64_t n_p2, const int32_t* __restrict__ nat2int,
                                                    const T* __restrict__ src, const double* __restrict__ ubc,
                                                    double* __restrict__ dst, int bnd_fill) {
  GRID_STRIDE_ROWS(nat, n_p2) {
    const int64_t k = nat2int[nat];
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int64_t o = ((int64_t)r * D + d) * n_p2 + nat;
        if (k >= 0) dst[o] = (double)src[(k * NRB + r) * D + d];
        else if (bnd_fill) dst[o] = ubc ? ubc[o] : 0.0;
      }
  }
}

// caller [nrb][n_p1] <-> internal [n_p1][nrb]
template <typename T, int NRB>
__global__ __launch_bounds__(kBlock) void k_p_in(int64_t n_p1, const double* __restrict__ src, T* __restrict__ dst) {
  GRID_STRIDE_ROWS(row, n_p1) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) dst[row * NRB + r] = (T)src[(int64_t)r * n_p1 + row];
  }
}
template <typename T, int NRB>
__global__ __launch_bounds__(kBlock) void k_p_out(int64_t n_p1, const T* __restrict__ src, double* __restrict__ dst) {
  GRID_STRIDE_ROWS(row, n_p1) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) dst[(int64_t)r * n_p1 + row] = (double)src[row * NRB + r];
  }
}

// ------------------------------------------------- right-hand side (FP64)

// Boundary columns of the load vector and the lifting, on the interior rows
// that touch the boundary: F[row] += sum_{c in Gamma} (M_ic f_c - A_ic G_c)
// (the interior columns of M f come from the sliced-ELL mass product).
constexpr int kRhsLanes = 4;

template <int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_rhs_bnd(int64_t nbc, int64_t n_p2, const int32_t* __restrict__ rows,
                                                    const int32_t* __restrict__ ptr, const int32_t* __restrict__ cols,
                                                    const int32_t* __restrict__ src, const double* __restrict__ M,
                                                    const double* __restrict__ L, const double* __restrict__ Dg,
                                                    double alpha, double mu, const double* __restrict__ f,
                                                    const double* __restrict__ ubc, double* __restrict__ F) {
  // kRhsLanes lanes per row take every kRhsLanes-th boundary column and add
  // their sums by lane exchanges (the lanes of a row share a wavefront)
  constexpr int W = D * NRB;
  GRID_STRIDE_ROWS_G(q, sub, nbc, kRhsLanes) {
    double acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    for (int32_t k = ptr[q] + sub; k < ptr[q + 1]; k += kRhsLanes) {
      const int64_t c = cols[k];
      const int64_t e = src[k];
      const double m = M[e];
      const double a = alpha * m + mu * L[e];
#pragma unroll
      for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int64_t o = ((int64_t)r * D + d) * n_p2 + c;
          double v = f ? m * f[o] : 0.0;
          if (ubc) {
            v -= a * ubc[o];
            if (Dg)  // strain form: mu sum_b D[d][b] G_b
              for (int b = 0; b < D; ++b) v -= mu * Dg[e * D * D + d * D + b] * ubc[((int64_t)r * D + b) * n_p2 + c];
          }
          acc[r * D + d] += v;
        }
    }
#pragma unroll
    for (int o = kRhsLanes / 2; o >= 1; o /= 2)
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] += __shfl_xor(acc[w], o);
    if (sub == 0) {
      const int64_t row = rows[q];
#pragma unroll
      for (int w = 0; w < W; ++w) F[row * W + w] += acc[w];
    }
  }
}

// g = -B_Gamma G over the P1 rows (CSR over all P2 columns, D planes)
template <int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_rhs_p(int64_t n_p1, int64_t n_p2, const int32_t* __restrict__ nat2int,
                                                  const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                  const double* __restrict__ Bv, const double* __restrict__ ubc,
                                                  double* __restrict__ g) {
  GRID_STRIDE_ROWS(row, n_p1) {
    double acc[NRB];
#pragma unroll
    for (int r = 0; r < NRB; ++r) acc[r] = 0;
    if (ubc) {
      for (int64_t k = rp[row]; k < rp[row + 1]; ++k) {
        const int64_t c = cols[k];
        if (nat2int[c] >= 0) continue;
#pragma unroll
        for (int r = 0; r < NRB; ++r)
#pragma unroll
          for (int d = 0; d < D; ++d) acc[r] -= Bv[k * D + d] * ubc[((int64_t)r * D + d) * n_p2 + c];
      }
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r) g[row * NRB + r] = acc[r];
  }
}

// Gradient pieces of the adjoint (FP64, CSR over all P2 nodes):
// dJdf[r][d][nat] = sum_k M[k] lam[int(col_k)]   (zero outside the interior)
template <int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_adj_dJdf(int64_t n_p2, const int32_t* __restrict__ nat2int,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                     const double* __restrict__ M, const double* __restrict__ lam,
                                                     double* __restrict__ out) {
  constexpr int W = D * NRB;
  GRID_STRIDE_ROWS(nat, n_p2) {
    double acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    for (int64_t k = rp[nat]; k < rp[nat + 1]; ++k) {
      const int64_t c = nat2int[cols[k]];
      if (c < 0) continue;
      const double m = M[k];
#pragma unroll
      for (int w = 0; w < W; ++w) acc[w] += m * lam[c * W + w];
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int d = 0; d < D; ++d) out[((int64_t)r * D + d) * n_p2 + nat] = acc[r * D + d];
  }
}

// dJdmu[r] = -sum_{interior rows} lam[row][r][:] . (L u_full)[row][r][:]
template <int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_adj_dJdmu(int64_t n_int, int64_t n_p2, const int32_t* __restrict__ int2nat,
                                                      const int32_t* __restrict__ rp, const int32_t* __restrict__ cols,
                                                      const double* __restrict__ L, const double* __restrict__ Dg,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ lam, double* res, double* partials) {
  constexpr int W = D * NRB;
  double part[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) part[r] = 0;
  GRID_STRIDE_ROWS(row, n_int) {
    const int64_t nat = int2nat[row];
    double acc[W];
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = 0;
    for (int64_t k = rp[nat]; k < rp[nat + 1]; ++k) {
      const int64_t c = cols[k];
      const double l = L[k];
#pragma unroll
      for (int r = 0; r < NRB; ++r)
#pragma unroll
        for (int d = 0; d < D; ++d) {
          double t = l * u[((int64_t)r * D + d) * n_p2 + c];
          if (Dg)  // strain form: the viscous matrix is L + D
            for (int b = 0; b < D; ++b) t += Dg[k * D * D + d * D + b] * u[((int64_t)r * D + b) * n_p2 + c];
          acc[r * D + d] += t;
        }
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r)
#pragma unroll
      for (int d = 0; d < D; ++d) part[r] -= lam[row * W + r * D + d] * acc[r * D + d];
  }
  grid_reduce<NRB>(part, partials);
}

}  // namespace stokes

namespace stokes {

// ------------------------------------------- coupled-vector (FGMRES) kernels
// A coupled vector is the velocity part [n_int][NRB][D] followed by the
// pressure part [n_p1][NRB]; right-hand side r owns slots r*D..r*D+D-1 of a
// velocity row and slot r of a pressure row.

struct Coef8 {
  double v[8];
};

// Both kernels map NRB lanes to one row (lane `sub` = right-hand side sub),
// so the lanes of a row read its W contiguous values together.

// Sum over the lanes of a wavefront that share lane mod G (G a power of two
// up to 64); lanes 0..G-1 then hold the G sums.
template <int G>
__device__ __forceinline__ double wave_sum_strided(double x) {
#pragma unroll
  for (int off = 32; off >= G; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

constexpr int kMdotChunk = 8;  // basis vectors per pass over w

// Partial dots h[j][r] = V_j . w for the basis vectors j of chunk blockIdx.y
// (kMdotChunk at a time, so w is read once per chunk): block partials to
// part[((chunk * gridDim.x + block) * kMdotChunk + j) * NRB + r].
template <typename TV, typename TW, int D, int NRB>
__global__ __launch_bounds__(kBlock) void k_mdot(int64_t n_int, int64_t n_p1, const TV* __restrict__ V, int64_t ldv,
                                                 int nb, const TW* __restrict__ w, double* __restrict__ part) {
  constexpr int W = D * NRB, CH = kMdotChunk;
  const int sub = (int)(threadIdx.x % NRB);
  const int j0 = blockIdx.y * CH;
  const int nj = nb - j0 < CH ? nb - j0 : CH;
  const int64_t nv = n_int * W;
  double acc[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) acc[j] = 0;
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / NRB; t < n_int + n_p1;
       t += (int64_t)gridDim.x * blockDim.x / NRB) {
    if (t < n_int) {
      const int64_t o = t * W + sub * D;
      double wv[D];
#pragma unroll
      for (int d = 0; d < D; ++d) wv[d] = (double)w[o + d];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        if (j < nj) {
          const TV* v = V + (int64_t)(j0 + j) * ldv + o;
          double s = 0;
#pragma unroll
          for (int d = 0; d < D; ++d) s += (double)v[d] * wv[d];
          acc[j] += s;
        }
      }
    } else {
      const int64_t o = nv + (t - n_int) * NRB + sub;
      const double wv = (double)w[o];
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (j < nj) acc[j] += (double)V[(int64_t)(j0 + j) * ldv + o] * wv;
    }
  }
  __shared__ double sh[kBlock / 64][CH][NRB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const double s = wave_sum_strided<NRB>(acc[j]);
    if (lane < NRB) sh[wave][j][lane] = s;
  }
  __syncthreads();
  if (threadIdx.x < CH * NRB) {
    const int j = threadIdx.x / NRB, r = threadIdx.x % NRB;
    double s = 0;
    for (int q = 0; q < kBlock / 64; ++q) s += sh[q][j][r];
    part[(((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * CH + j) * NRB + r] = s;
  }
}

// h[i][r] = sum over blocks of the partials of basis vector i (one block per
// i, fixed order)
template <int NRB>
__global__ __launch_bounds__(kBlock) void k_mdot_fin(int nblk, const double* __restrict__ part, double* __restrict__ h) {
  const int i = blockIdx.x, ch = i / kMdotChunk, j = i % kMdotChunk;
  double acc[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) acc[r] = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int r = 0; r < NRB; ++r) acc[r] += part[(((int64_t)ch * nblk + b) * kMdotChunk + j) * NRB + r];
  __shared__ double tot[NRB];
  block_sum<NRB>(acc, tot);
  if (threadIdx.x < NRB) h[i * NRB + threadIdx.x] = tot[threadIdx.x];
}

// w += sgn * sum_{i<nb} h[i][r] V_i (accumulated in FP64, stored in TW);
// NORM: res[r] = ||w_r||^2 of the stored values
// sig2 (optional): per basis vector and right-hand side, a factor on h (the
// squared scale of a basis stored unnormalized); wf (optional): the stored w
// again, rounded to TF.
template <typename TV, typename TW, int D, int NRB, int NORM, typename TF = TW>
__global__ __launch_bounds__(kBlock) void k_mupdate(int64_t n_int, int64_t n_p1, const TV* __restrict__ V,
                                                    int64_t ldv, int nb, const double* __restrict__ h, double sgn,
                                                    TW* __restrict__ w, double* res, double* partials,
                                                    const double* __restrict__ sig2 = nullptr,
                                                    TF* __restrict__ wf = nullptr) {
  constexpr int W = D * NRB;
  __shared__ double hs[64 * NRB];
  for (int i = threadIdx.x; i < nb * NRB; i += blockDim.x) hs[i] = sgn * h[i] * (sig2 ? sig2[i] : 1.0);
  __syncthreads();
  const int sub = (int)(threadIdx.x % NRB);
  const int64_t nv = n_int * W;
  double part = 0;
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / NRB; t < n_int + n_p1;
       t += (int64_t)gridDim.x * blockDim.x / NRB) {
    if (t < n_int) {
      const int64_t o = t * W + sub * D;
      double a[D];
#pragma unroll
      for (int d = 0; d < D; ++d) a[d] = (double)w[o + d];
      for (int i = 0; i < nb; ++i) {
        const TV* v = V + (int64_t)i * ldv + o;
        const double hi = hs[i * NRB + sub];
#pragma unroll
        for (int d = 0; d < D; ++d) a[d] += hi * (double)v[d];
      }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const TW st = (TW)a[d];
        w[o + d] = st;
        if (wf) wf[o + d] = (TF)st;
        if (NORM) part += (double)st * (double)st;
      }
    } else {
      const int64_t o = nv + (t - n_int) * NRB + sub;
      double a = (double)w[o];
      for (int i = 0; i < nb; ++i) a += hs[i * NRB + sub] * (double)V[(int64_t)i * ldv + o];
      const TW st = (TW)a;
      w[o] = st;
      if (wf) wf[o] = (TF)st;
      if (NORM) part += (double)st * (double)st;
    }
  }
  if (NORM) {
    double pf[NRB];
#pragma unroll
    for (int r = 0; r < NRB; ++r) pf[r] = r == sub ? part : 0.0;
    grid_reduce<NRB>(pf, partials);
  }
}

// First Gram-Schmidt update fused with the second pass's dot products:
//   w <- w - sum_{i<nb} h[i][r] V_i   (FP64 sums, stored in TW), then
//   partial dots V_i . w of the stored w, for i < nb <= kFusedMax,
// written in k_mdot's partial layout (chunk i / 8, slot i mod 8) with the same
// row mapping and block reduction, so k_mdot_fin gives the same sums as a
// separate k_mdot pass.  One read of the basis instead of two.  w is read
// from win (TI, may be w itself) and written in TW.
// GRAM = 1 (the update with the whole CGS2 coefficients, the new basis
// column): also ||w||^2 of the stored w as entry nb (chunk nb / 8, slot
// nb mod 8), and wf (optional) receives w rounded to TF.  NM: the largest nb
// (the basis values of a row are held in registers for the dots); launched
// with 8 up to 8 columns and 16 beyond, up to kFusedMax.
constexpr int kFusedMax = 16;
template <typename TV, typename TW, int D, int NRB, typename TI = TW, int GRAM = 0, typename TF = TW, int NM = 8>
__global__ __launch_bounds__(kBlock) void k_mupdate_dot(int64_t n_int, int64_t n_p1, const TV* __restrict__ V,
                                                        int64_t ldv, int nb, const double* __restrict__ h,
                                                        const TI* win, TW* w, double* __restrict__ part,
                                                        const double* __restrict__ sig2 = nullptr,
                                                        TF* __restrict__ wf = nullptr) {
  constexpr int W = D * NRB, CH = kMdotChunk, NA = NM + GRAM;
  __shared__ double hs[NM * NRB];
  for (int i = threadIdx.x; i < nb * NRB; i += blockDim.x) hs[i] = -h[i] * (sig2 ? sig2[i] : 1.0);
  __syncthreads();
  const int sub = (int)(threadIdx.x % NRB);
  const int64_t nv = n_int * W;
  double acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0;
  for (int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / NRB; t < n_int + n_p1;
       t += (int64_t)gridDim.x * blockDim.x / NRB) {
    if (t < n_int) {
      const int64_t o = t * W + sub * D;
      double a[D];
      TV v[NM][D];
#pragma unroll
      for (int d = 0; d < D; ++d) a[d] = (double)win[o + d];
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) {
#pragma unroll
          for (int d = 0; d < D; ++d) v[i][d] = V[(int64_t)i * ldv + o + d];
        }
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) {
          const double hi = hs[i * NRB + sub];
#pragma unroll
          for (int d = 0; d < D; ++d) a[d] += hi * (double)v[i][d];
        }
      double st[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const TW sv = (TW)a[d];
        w[o + d] = sv;
        if (GRAM && wf) wf[o + d] = (TF)sv;
        st[d] = (double)sv;
      }
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) {
          double sacc = 0;
#pragma unroll
          for (int d = 0; d < D; ++d) sacc += (double)v[i][d] * st[d];
          acc[i] += sacc;
        }
      if constexpr (GRAM) {
        double nacc = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) nacc += st[d] * st[d];
        acc[NM] += nacc;
      }
    } else {
      const int64_t o = nv + (t - n_int) * NRB + sub;
      TV v[NM];
      double a = (double)win[o];
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) v[i] = V[(int64_t)i * ldv + o];
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) a += hs[i * NRB + sub] * (double)v[i];
      const TW sv = (TW)a;
      w[o] = sv;
      if (GRAM && wf) wf[o] = (TF)sv;
#pragma unroll
      for (int i = 0; i < NM; ++i)
        if (i < nb) acc[i] += (double)v[i] * (double)sv;
      if constexpr (GRAM) acc[NM] += (double)sv * (double)sv;
    }
  }
  __shared__ double sh[kBlock / 64][NA][NRB];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const double sv = wave_sum_strided<NRB>(acc[i]);
    if (lane < NRB) sh[wave][i][lane] = sv;
  }
  __syncthreads();
  // entries 0 .. nb-1: the dots; entry nb (GRAM): the squared norm (slot NM of sh)
  for (int q = threadIdx.x; q < (nb + GRAM) * NRB; q += blockDim.x) {
    const int i = q / NRB, r = q % NRB;
    const int si = i < nb ? i : NM;
    double sv = 0;
    for (int k = 0; k < kBlock / 64; ++k) sv += sh[k][si][r];
    part[((((int64_t)(i / CH)) * gridDim.x + blockIdx.x) * CH + (i % CH)) * NRB + r] = sv;
  }
}

// CGS2 with the second projection from the Gram matrix of the (unnormalized)
// basis columns C_i, R_ik = C_i . C_k, kept per right-hand side: with the
// first projection's dots a_i = C_i . w and the squared scales s_i^2 of the
// columns, the second projection's dots are
//   b_i = C_i . (w - sum_k s_k^2 a_k C_k) = a_i - sum_k R_ik s_k^2 a_k,
// so one update w <- w - sum_i s_i^2 (a_i + b_i) C_i gives the CGS2 vector
// without a second pass over the basis.  One block; writes b (h2) and a + b
// (hsum).  R: [i][k][r] with strides 64 * 8 and 8.
constexpr int kGramLd = 64;
template <int NRB>
__global__ __launch_bounds__(kBlock) void k_gram_h2(int nb, const double* __restrict__ R,
                                                    const double* __restrict__ sig2, const double* __restrict__ h1,
                                                    double* __restrict__ h2, double* __restrict__ hsum) {
  for (int q = threadIdx.x; q < nb * NRB; q += blockDim.x) {
    const int i = q / NRB, r = q % NRB;
    double s = 0;
    for (int k = 0; k < nb; ++k) s += R[((int64_t)i * kGramLd + k) * 8 + r] * sig2[k * NRB + r] * h1[k * NRB + r];
    const double b = h1[i * NRB + r] - s;
    h2[i * NRB + r] = b;
    hsum[i * NRB + r] = h1[i * NRB + r] + b;
  }
}

// The new column's Gram row from k_mupdate_dot<GRAM = 1>'s partials: entry
// i < nb is C_i . C_nb, entry nb is ||C_nb||^2 (also written to nrm[r]).
// One block per entry.
template <int NRB>
__global__ __launch_bounds__(kBlock) void k_gram_fin(int nblk, const double* __restrict__ part, int nb,
                                                     double* __restrict__ R, double* __restrict__ nrm) {
  const int i = blockIdx.x, ch = i / kMdotChunk, j = i % kMdotChunk;
  double acc[NRB];
#pragma unroll
  for (int r = 0; r < NRB; ++r) acc[r] = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int r = 0; r < NRB; ++r) acc[r] += part[(((int64_t)ch * nblk + b) * kMdotChunk + j) * NRB + r];
  __shared__ double tot[NRB];
  block_sum<NRB>(acc, tot);
  if (threadIdx.x < NRB) {
    const int r = threadIdx.x;
    const double v = tot[r];
    R[((int64_t)i * kGramLd + nb) * 8 + r] = v;
    R[((int64_t)nb * kGramLd + i) * 8 + r] = v;
    if (i == nb) nrm[r] = v;
  }
}

// v = s[r] * w  (coupled vectors, per right-hand-side scale); vf (optional)
// receives the same values rounded to TF
template <typename TS, int D, int NRB, typename TF = TS>
__global__ __launch_bounds__(kBlock) void k_scale_coupled(int64_t n_int, int64_t n_p1, Coef8 s,
                                                          const TS* __restrict__ w, TS* __restrict__ v,
                                                          TF* __restrict__ vf) {
  constexpr int W = D * NRB;
  const int64_t nv = n_int * W;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv + n_p1 * NRB;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = i < nv ? (int)((i % W) / D) : (int)((i - nv) % NRB);
    const TS x = (TS)(s.v[r] * (double)w[i]);
    v[i] = x;
    if (vf) vf[i] = (TF)x;
  }
}

// y = a[r] x + b[r] y over rows of WROW values, r = slot / CPS
template <typename TX, typename TY, int WROW, int CPS>
__global__ __launch_bounds__(kBlock) void k_axpy_rhs(int64_t nrows, Coef8 a, Coef8 b, const TX* __restrict__ x,
                                                     TY* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrows * WROW;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i % WROW) / CPS;
    y[i] = (TY)(a.v[r] * (double)x[i] + b.v[r] * (double)y[i]);
  }
}

// ------------------------------------------------------ scalar bookkeeping

// Start of a CG: bb from slot sums, tolerances, flags.
static __global__ void k_scal_init(Scalars* sc, const double* __restrict__ slots, int cps, int nsys, double rtol2) {
  const int s = threadIdx.x;
  if (s < kMaxSys) {
    double bb = 0;
    if (s < nsys)
      for (int w = s * cps; w < (s + 1) * cps; ++w) bb += slots[w];
    sc->bb[s] = bb;
    sc->tol2[s] = rtol2 * bb;
    sc->rr[s] = bb;
    sc->active[s] = (s < nsys && bb > 0) ? 1 : 0;
    sc->rho[s] = sc->rho_old[s] = sc->alpha[s] = sc->beta[s] = sc->sigma[s] = 0;
  }
  if (s == 0) sc->breakdown = 0;
}

// rho from slot sums; beta = rho / rho_prev (0 on the first step)
static __global__ void k_scal_rho(Scalars* sc, const double* __restrict__ slots, int cps, int nsys, int first) {
  const int s = threadIdx.x;
  if (s < nsys) {
    double rho = 0;
    for (int w = s * cps; w < (s + 1) * cps; ++w) rho += slots[w];
    sc->beta[s] = (!first && sc->active[s] && sc->rho[s] != 0) ? rho / sc->rho[s] : 0.0;
    if (sc->active[s] && !(rho > 0)) sc->breakdown = 1;
    sc->rho[s] = rho;
  }
}

// g = -(g - m sum_r / (1^T m)): the transpose of the zero-integral
// normalisation applied to a pressure loss gradient, negated for the forward form
template <int NRB>
__global__ __launch_bounds__(kBlock) void k_adj_jp(int64_t n_p1, const double* __restrict__ m,
                                                   const double* __restrict__ sum, double inv_msum,
                                                   double* __restrict__ g) {
  GRID_STRIDE_ROWS(row, n_p1) {
#pragma unroll
    for (int r = 0; r < NRB; ++r) g[row * NRB + r] = -(g[row * NRB + r] - m[row] * sum[r] * inv_msum);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set(int64_t n, T v, T* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

}  // namespace stokes

// Host-side Kuhn mesh, numbering and sparsity patterns (see mesh_host.h).
#include "mesh_host.h"

#include <algorithm>
#include <thread>

namespace stokes {

int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

namespace {

uint64_t splitmix_finalise(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// U in [0, 1): top 53 bits of the finalised counter state.
double unit_draw(uint64_t seed, uint64_t counter) {
  const uint64_t state = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  return static_cast<double>(splitmix_finalise(state) >> 11) * 0x1.0p-53;
}

template <class F>
void parallel_for(int64_t n, F&& body) {
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (nt > 16) nt = 16;
  if (n < 4096) nt = 1;
  if (nt == 1) {
    body(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min<int64_t>(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&body, b, e] { body(b, e); });
  }
  for (auto& x : th) x.join();
}

}  // namespace

bool build_mesh(int dim, int n, uint64_t seed, double jitter, HostMesh& m, int order) {
  m.dim = dim;
  m.n = n;
  m.nloc = dim == 3 ? 10 : 6;
  const int nv = dim + 1;
  const int64_t n1 = n + 1, n2 = 2 * int64_t(n) + 1;
  m.n_p1 = ipow(n1, dim);
  m.n_p2 = ipow(n2, dim);
  const int64_t ncell = ipow(n, dim);
  const int nperm = dim == 3 ? 6 : 2;
  m.n_e = ncell * nperm;
  if (m.n_p2 >= (int64_t(1) << 31) || m.n_e >= (int64_t(1) << (31 - kLocBits))) return false;
  if (order == 3 && ipow(3 * int64_t(n) + 1, dim) >= (int64_t(1) << 31)) return false;

  // vertex coordinates: x fastest, interior vertices jittered
  m.vcoords.assign(m.n_p1 * dim, 0.0);
  const double inv_n_div = static_cast<double>(n);
  for (int64_t g = 0; g < m.n_p1; ++g) {
    int64_t rem = g;
    int idx[3] = {0, 0, 0};
    bool interior = true;
    for (int c = 0; c < dim; ++c) {
      idx[c] = static_cast<int>(rem % n1);
      rem /= n1;
      if (idx[c] == 0 || idx[c] == n) interior = false;
    }
    for (int c = 0; c < dim; ++c) {
      double x = static_cast<double>(idx[c]);
      if (interior) {
        const double u = unit_draw(seed, static_cast<uint64_t>(dim) * g + c);
        const double two_u = 2.0 * u;
        const double centred = two_u - 1.0;
        const double delta = centred * jitter;
        x = x + delta;
      }
      m.vcoords[g * dim + c] = x / inv_n_div;
    }
  }

  // simplices (cell-major, x fastest, then permutations in lexicographic order)
  static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  static const int perm2[2][2] = {{0, 1}, {1, 0}};
  static const int edges3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  static const int edges2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  m.elems.assign(m.n_e * nv, 0);
  m.p2.assign(m.n_e * m.nloc, 0);
  int64_t e = 0;
  for (int64_t cell = 0; cell < ncell; ++cell) {
    int64_t rem = cell;
    int cg[3] = {0, 0, 0};
    for (int c = 0; c < dim; ++c) {
      cg[c] = static_cast<int>(rem % n);
      rem /= n;
    }
    for (int q = 0; q < nperm; ++q, ++e) {
      int pos[4][3];
      for (int c = 0; c < 3; ++c) pos[0][c] = cg[c];
      for (int s = 0; s < dim; ++s) {
        for (int c = 0; c < 3; ++c) pos[s + 1][c] = pos[s][c];
        const int ax = dim == 3 ? perm3[q][s] : perm2[q][s];
        pos[s + 1][ax] += 1;
      }
      for (int a = 0; a < nv; ++a) {
        int64_t id = 0, st = 1;
        for (int c = 0; c < dim; ++c, st *= n1) id += pos[a][c] * st;
        m.elems[e * nv + a] = static_cast<int32_t>(id);
        int64_t id2 = 0, st2 = 1;
        for (int c = 0; c < dim; ++c, st2 *= n2) id2 += 2 * pos[a][c] * st2;
        m.p2[e * m.nloc + a] = static_cast<int32_t>(id2);
      }
      const int ned = dim == 3 ? 6 : 3;
      for (int k = 0; k < ned; ++k) {
        const int a = dim == 3 ? edges3[k][0] : edges2[k][0];
        const int b = dim == 3 ? edges3[k][1] : edges2[k][1];
        int64_t id2 = 0, st2 = 1;
        for (int c = 0; c < dim; ++c, st2 *= n2) id2 += (pos[a][c] + pos[b][c]) * st2;
        m.p2[e * m.nloc + nv + k] = static_cast<int32_t>(id2);
      }
    }
  }

  // P2 coordinates: vertices copy, edge nodes (x_a + x_b) * 0.5
  m.p2coords.assign(m.n_p2 * dim, 0.0);
  for (int64_t el = 0; el < m.n_e; ++el) {
    const int32_t* ev = &m.elems[el * nv];
    const int32_t* ep = &m.p2[el * m.nloc];
    for (int a = 0; a < nv; ++a)
      for (int c = 0; c < dim; ++c) m.p2coords[int64_t(ep[a]) * dim + c] = m.vcoords[int64_t(ev[a]) * dim + c];
    const int ned = dim == 3 ? 6 : 3;
    for (int k = 0; k < ned; ++k) {
      const int a = dim == 3 ? edges3[k][0] : edges2[k][0];
      const int b = dim == 3 ? edges3[k][1] : edges2[k][1];
      for (int c = 0; c < dim; ++c) {
        const double s = m.vcoords[int64_t(ev[a]) * dim + c] + m.vcoords[int64_t(ev[b]) * dim + c];
        m.p2coords[int64_t(ep[nv + k]) * dim + c] = s * 0.5;
      }
    }
  }

  m.p2_bnd.assign(m.n_p2, 0);
  for (int64_t id = 0; id < m.n_p2; ++id) {
    int64_t rem = id;
    for (int c = 0; c < dim; ++c) {
      const int64_t I = rem % n2;
      rem /= n2;
      if (I == 0 || I == n2 - 1) m.p2_bnd[id] = 1;
    }
  }
  m.order = order;
  if (order != 3) {
    // P2/P1: the pressure lives on the vertices
    m.q = m.elems;
    m.n_q = m.n_p1;
    m.nqloc = nv;
    return true;
  }
  // P3/P2: the P2 nodes above become the pressure space; the velocity moves
  // to the P3 nodes of the (3n+1)^d lattice
  m.q.swap(m.p2);
  m.n_q = m.n_p2;
  m.nqloc = m.nloc;
  const int64_t n3 = 3 * int64_t(n) + 1;
  m.n_p2 = ipow(n3, dim);
  const int nf = dim == 3 ? 4 : 1;
  static const int faces3[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
  static const int faces2[1][3] = {{0, 1, 2}};
  const int ned = dim == 3 ? 6 : 3;
  m.nloc = nv + 2 * ned + nf;
  m.p2.assign(m.n_e * m.nloc, 0);
  m.p2coords.assign(m.n_p2 * dim, 0.0);
  for (int64_t el = 0; el < m.n_e; ++el) {
    const int32_t* ev = &m.elems[el * nv];
    int32_t* out = &m.p2[el * m.nloc];
    // lattice position (units h / 3) of vertex a of this simplex
    auto vpos = [&](int a, int c) { return static_cast<int64_t>((ev[a] / ipow(n1, c)) % n1); };
    auto node_id = [&](const int* cm) {
      int64_t id = 0, st = 1;
      for (int c = 0; c < dim; ++c, st *= n3) {
        int64_t x = 0;
        for (int a = 0; a < nv; ++a) x += cm[a] * vpos(a, c);
        id += x * st;
      }
      return id;
    };
    auto X = [&](int a, int c) { return m.vcoords[int64_t(ev[a]) * dim + c]; };
    int li = 0;
    for (int a = 0; a < nv; ++a, ++li) {
      int cm[4] = {0, 0, 0, 0};
      cm[a] = 3;
      const int64_t id = node_id(cm);
      out[li] = static_cast<int32_t>(id);
      for (int c = 0; c < dim; ++c) m.p2coords[id * dim + c] = X(a, c);
    }
    for (int k = 0; k < ned; ++k) {
      const int a = dim == 3 ? edges3[k][0] : edges2[k][0];
      const int b = dim == 3 ? edges3[k][1] : edges2[k][1];
      for (int side = 0; side < 2; ++side, ++li) {
        const int near = side == 0 ? a : b, far = side == 0 ? b : a;
        int cm[4] = {0, 0, 0, 0};
        cm[near] = 2;
        cm[far] = 1;
        const int64_t id = node_id(cm);
        out[li] = static_cast<int32_t>(id);
        for (int c = 0; c < dim; ++c) {
          const double twice = 2.0 * X(near, c);
          const double s = twice + X(far, c);
          m.p2coords[id * dim + c] = s / 3.0;
        }
      }
    }
    for (int k = 0; k < nf; ++k, ++li) {
      const int* f = dim == 3 ? faces3[k] : faces2[k];
      int cm[4] = {0, 0, 0, 0};
      for (int t = 0; t < 3; ++t) cm[f[t]] = 1;
      const int64_t id = node_id(cm);
      out[li] = static_cast<int32_t>(id);
      int s3[3] = {f[0], f[1], f[2]};  // local indices sorted by global vertex id
      std::sort(s3, s3 + 3, [&](int x, int y) { return ev[x] < ev[y]; });
      for (int c = 0; c < dim; ++c) {
        const double s01 = X(s3[0], c) + X(s3[1], c);
        const double s = s01 + X(s3[2], c);
        m.p2coords[id * dim + c] = s / 3.0;
      }
    }
  }
  m.p2_bnd.assign(m.n_p2, 0);
  for (int64_t id = 0; id < m.n_p2; ++id) {
    int64_t rem = id;
    for (int c = 0; c < dim; ++c) {
      const int64_t I = rem % n3;
      rem /= n3;
      if (I == 0 || I == n3 - 1) m.p2_bnd[id] = 1;
    }
  }
  return true;
}

void incidence(const std::vector<int32_t>& nodes, int nl, int64_t n_e, int64_t n_nodes,
               std::vector<int64_t>& ptr, std::vector<int32_t>& list) {
  ptr.assign(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_e; ++e)
    for (int a = 0; a < nl; ++a) ptr[nodes[e * nl + a] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) ptr[i + 1] += ptr[i];
  list.assign(ptr[n_nodes], 0);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t e = 0; e < n_e; ++e)
    for (int a = 0; a < nl; ++a) list[fill[nodes[e * nl + a]]++] = static_cast<int32_t>((e << kLocBits) | a);
}

void element_pattern(const std::vector<int32_t>& row_nodes, int nr, int64_t nrows,
                     const std::vector<int32_t>& col_nodes, int nc, int64_t ncols, int64_t n_e,
                     HostCsr& out) {
  std::vector<int64_t> iptr;
  std::vector<int32_t> ilist;
  incidence(row_nodes, nr, n_e, nrows, iptr, ilist);
  out.nrows = nrows;
  out.ncols = ncols;
  out.rowptr.assign(nrows + 1, 0);
  auto gather = [&](int64_t r, std::vector<int32_t>& buf) {
    buf.clear();
    for (int64_t k = iptr[r]; k < iptr[r + 1]; ++k) {
      const int64_t e = ilist[k] >> kLocBits;
      for (int b = 0; b < nc; ++b) buf.push_back(col_nodes[e * nc + b]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
  };
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    std::vector<int32_t> buf;
    for (int64_t r = b; r < e; ++r) {
      gather(r, buf);
      out.rowptr[r + 1] = static_cast<int64_t>(buf.size());
    }
  });
  for (int64_t r = 0; r < nrows; ++r) out.rowptr[r + 1] += out.rowptr[r];
  out.cols.assign(out.rowptr[nrows], 0);
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    std::vector<int32_t> buf;
    for (int64_t r = b; r < e; ++r) {
      gather(r, buf);
      std::copy(buf.begin(), buf.end(), out.cols.begin() + out.rowptr[r]);
    }
  });
}

void restrict_pattern(const HostCsr& in, const std::vector<int32_t>& row_map, int64_t nrows_out,
                      const std::vector<int32_t>& col_map, int64_t ncols_out, HostCsr& out,
                      std::vector<int64_t>* src) {
  out.nrows = nrows_out;
  out.ncols = ncols_out;
  out.rowptr.assign(nrows_out + 1, 0);
  std::vector<int64_t> inrow(nrows_out, -1);
  for (int64_t r = 0; r < in.nrows; ++r)
    if (row_map[r] >= 0) inrow[row_map[r]] = r;
  parallel_for(nrows_out, [&](int64_t b, int64_t e) {
    for (int64_t ro = b; ro < e; ++ro) {
      const int64_t r = inrow[ro];
      int64_t cnt = 0;
      for (int64_t k = in.rowptr[r]; k < in.rowptr[r + 1]; ++k)
        if (col_map[in.cols[k]] >= 0) ++cnt;
      out.rowptr[ro + 1] = cnt;
    }
  });
  for (int64_t r = 0; r < nrows_out; ++r) out.rowptr[r + 1] += out.rowptr[r];
  out.cols.assign(out.rowptr[nrows_out], 0);
  if (src) src->assign(out.rowptr[nrows_out], 0);
  parallel_for(nrows_out, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, int64_t>> buf;
    for (int64_t ro = b; ro < e; ++ro) {
      const int64_t r = inrow[ro];
      buf.clear();
      for (int64_t k = in.rowptr[r]; k < in.rowptr[r + 1]; ++k) {
        const int32_t c = col_map[in.cols[k]];
        if (c >= 0) buf.emplace_back(c, k);
      }
      std::sort(buf.begin(), buf.end());
      int64_t o = out.rowptr[ro];
      for (auto& pr : buf) {
        out.cols[o] = pr.first;
        if (src) (*src)[o] = pr.second;
        ++o;
      }
    }
  });
}

void transpose_pattern(const HostCsr& in, HostCsr& out, std::vector<int64_t>& src) {
  out.nrows = in.ncols;
  out.ncols = in.nrows;
  out.rowptr.assign(out.nrows + 1, 0);
  for (int64_t k = 0; k < in.rowptr[in.nrows]; ++k) out.rowptr[in.cols[k] + 1]++;
  for (int64_t r = 0; r < out.nrows; ++r) out.rowptr[r + 1] += out.rowptr[r];
  out.cols.assign(out.rowptr[out.nrows], 0);
  src.assign(out.rowptr[out.nrows], 0);
  std::vector<int64_t> fill(out.rowptr.begin(), out.rowptr.end() - 1);
  // rows of `in` visited in increasing order, so each transposed row is sorted
  for (int64_t r = 0; r < in.nrows; ++r)
    for (int64_t k = in.rowptr[r]; k < in.rowptr[r + 1]; ++k) {
      const int64_t o = fill[in.cols[k]]++;
      out.cols[o] = static_cast<int32_t>(r);
      src[o] = k;
    }
}

void product_pattern(const HostCsr& A, const HostCsr& At, const std::vector<int32_t>& mid_keep, HostCsr& out) {
  out.nrows = A.nrows;
  out.ncols = A.nrows;
  out.rowptr.assign(A.nrows + 1, 0);
  auto gather = [&](int64_t r, std::vector<int32_t>& buf) {
    buf.clear();
    for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k) {
      const int32_t j = A.cols[k];
      if (mid_keep[j] < 0) continue;
      for (int64_t t = At.rowptr[j]; t < At.rowptr[j + 1]; ++t) buf.push_back(At.cols[t]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
  };
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    std::vector<int32_t> buf;
    for (int64_t r = b; r < e; ++r) {
      gather(r, buf);
      out.rowptr[r + 1] = static_cast<int64_t>(buf.size());
    }
  });
  for (int64_t r = 0; r < A.nrows; ++r) out.rowptr[r + 1] += out.rowptr[r];
  out.cols.assign(out.rowptr[A.nrows], 0);
  parallel_for(A.nrows, [&](int64_t b, int64_t e) {
    std::vector<int32_t> buf;
    for (int64_t r = b; r < e; ++r) {
      gather(r, buf);
      std::copy(buf.begin(), buf.end(), out.cols.begin() + out.rowptr[r]);
    }
  });
}

void galerkin_p1(int dim, int nf, int nc, const HostCsr& A, const std::vector<double>& av, HostCsr& out,
                 std::vector<double>& ov) {
  const int64_t ncv = ipow(nc + 1, dim), nfv1 = nf + 1, ncv1 = nc + 1;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(ncv);
  parallel_for(ncv, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, double>> acc;
    for (int64_t I = b; I < e; ++I) {
      acc.clear();
      int G[3] = {0, 0, 0};
      int64_t rem = I;
      for (int d = 0; d < dim; ++d) {
        G[d] = static_cast<int>(rem % ncv1);
        rem /= ncv1;
      }
      // fine rows f with P[f, I] != 0: f = 2G (weight 1) and 2G +- s (weight 1/2)
      for (int s = 0; s < (1 << dim); ++s) {
        for (int sg = 1; sg >= -1; sg -= 2) {
          if (s == 0 && sg < 0) continue;
          int64_t f = 0, st = 1;
          bool ok = true;
          for (int d = 0; d < dim; ++d, st *= nfv1) {
            const int g = 2 * G[d] + sg * ((s >> d) & 1);
            ok = ok && g >= 0 && g <= nf;
            f += int64_t(g) * st;
          }
          if (!ok) continue;
          const double w = s == 0 ? 1.0 : 0.5;
          for (int64_t k = A.rowptr[f]; k < A.rowptr[f + 1]; ++k) {
            // column g of the fine level interpolates coarse vertices a and b
            int64_t rg = A.cols[k], a = 0, bb = 0, sc = 1;
            for (int d = 0; d < dim; ++d, sc *= ncv1) {
              const int64_t fg = rg % nfv1;
              rg /= nfv1;
              const int64_t par = fg & 1;
              a += ((fg - par) / 2) * sc;
              bb += ((fg + par) / 2) * sc;
            }
            const double v = 0.5 * w * av[k];
            acc.emplace_back(static_cast<int32_t>(a), v);
            acc.emplace_back(static_cast<int32_t>(bb), v);
          }
        }
      }
      std::stable_sort(acc.begin(), acc.end(),
                       [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                         return x.first < y.first;
                       });
      auto& row = rows[I];
      row.clear();
      for (const auto& pr : acc) {
        if (!row.empty() && row.back().first == pr.first) row.back().second += pr.second;
        else row.push_back(pr);
      }
    }
  });
  out.nrows = out.ncols = ncv;
  out.rowptr.assign(ncv + 1, 0);
  for (int64_t I = 0; I < ncv; ++I) out.rowptr[I + 1] = out.rowptr[I] + static_cast<int64_t>(rows[I].size());
  out.cols.resize(out.rowptr[ncv]);
  ov.resize(out.rowptr[ncv]);
  for (int64_t I = 0; I < ncv; ++I) {
    int64_t o = out.rowptr[I];
    for (const auto& pr : rows[I]) {
      out.cols[o] = pr.first;
      ov[o] = pr.second;
      ++o;
    }
  }
}

void p2_prolongation(int dim, int nf, const std::vector<int32_t>& fine_nat, HostCsr& P, std::vector<double>& pv) {
  const int nc = nf / 2;
  const int64_t n2f = 2 * int64_t(nf) + 1, n2c = 2 * int64_t(nc) + 1, nic = n2c - 2;
  const int64_t nrows = static_cast<int64_t>(fine_nat.size());
  auto coarse_index = [&](const int64_t* G) -> int64_t {  // interior index or -1 on the boundary
    int64_t idx = 0, st = 1;
    for (int d = 0; d < dim; ++d, st *= nic) {
      if (G[d] <= 0 || G[d] >= n2c - 1) return -1;
      idx += (G[d] - 1) * st;
    }
    return idx;
  };
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nrows);
  parallel_for(nrows, [&](int64_t b, int64_t e) {
    for (int64_t r = b; r < e; ++r) {
      int64_t F[3] = {0, 0, 0}, rem = fine_nat[r];
      for (int d = 0; d < dim; ++d) {
        F[d] = rem % n2f;
        rem /= n2f;
      }
      // coarse cell and local coordinates (quarters of the coarse cell)
      int64_t cell[3];
      double xi[3];
      for (int d = 0; d < dim; ++d) {
        cell[d] = std::min<int64_t>(F[d] / 4, nc - 1);
        xi[d] = double(F[d] - 4 * cell[d]) / 4.0;
      }
      // Kuhn simplex: axes by decreasing local coordinate (ties by axis)
      int pi[3] = {0, 1, 2};
      std::stable_sort(pi, pi + dim, [&](int a, int b2) { return xi[a] > xi[b2]; });
      double lam[4];
      lam[0] = 1.0 - xi[pi[0]];
      for (int a = 1; a < dim; ++a) lam[a] = xi[pi[a - 1]] - xi[pi[a]];
      lam[dim] = xi[pi[dim - 1]];
      int64_t v[4][3];
      for (int d = 0; d < dim; ++d) v[0][d] = cell[d];
      for (int a = 1; a <= dim; ++a) {
        for (int d = 0; d < dim; ++d) v[a][d] = v[a - 1][d];
        v[a][pi[a - 1]] += 1;
      }
      auto& row = rows[r];
      row.clear();
      auto add = [&](const int64_t* G, double w) {
        if (w == 0.0) return;
        const int64_t ci = coarse_index(G);
        if (ci >= 0) row.emplace_back(static_cast<int32_t>(ci), w);
      };
      for (int a = 0; a <= dim; ++a) {  // vertex functions lam (2 lam - 1) at node 2 v_a
        int64_t G[3];
        for (int d = 0; d < dim; ++d) G[d] = 2 * v[a][d];
        add(G, lam[a] * (2.0 * lam[a] - 1.0));
      }
      for (int a = 0; a <= dim; ++a)  // edge functions 4 lam_a lam_b at node v_a + v_b
        for (int b2 = a + 1; b2 <= dim; ++b2) {
          int64_t G[3];
          for (int d = 0; d < dim; ++d) G[d] = v[a][d] + v[b2][d];
          add(G, 4.0 * lam[a] * lam[b2]);
        }
      std::sort(row.begin(), row.end());
      size_t o = 0;
      for (size_t k = 0; k < row.size(); ++k) {
        if (o > 0 && row[o - 1].first == row[k].first) row[o - 1].second += row[k].second;
        else row[o++] = row[k];
      }
      row.resize(o);
    }
  });
  P.nrows = nrows;
  P.ncols = 1;
  for (int d = 0; d < dim; ++d) P.ncols *= nic;
  P.rowptr.assign(nrows + 1, 0);
  for (int64_t r = 0; r < nrows; ++r) P.rowptr[r + 1] = P.rowptr[r] + static_cast<int64_t>(rows[r].size());
  P.cols.resize(P.rowptr[nrows]);
  pv.resize(P.rowptr[nrows]);
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t o = P.rowptr[r];
    for (const auto& pr : rows[r]) {
      P.cols[o] = pr.first;
      pv[o] = pr.second;
      ++o;
    }
  }
}

}  // namespace stokes

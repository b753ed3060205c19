// Host-side structured Kuhn mesh, Taylor-Hood numbering and sparsity patterns.
//
// The mesh is the unit square / cube cut into n^d cells, each split into d!
// simplices (Kuhn split): for every permutation pi of the axes, taken in
// lexicographic order, the simplex (v0, v0 + e_pi0, v0 + e_pi0 + e_pi1, ...,
// v0 + (1,..,1)).  P2 nodes are the points of the refined (2n+1)^d grid
// (vertex v -> 2v, edge (a, b) -> v_a + v_b).  With the P3/P2 pair the
// velocity nodes are the points of the (3n+1)^d lattice (barycentric
// multi-index c, |c| = 3, of a simplex with vertex lattice points V_a -> the
// point sum c_a V_a) and the pressure nodes are the P2 points above; the local
// P3 order is vertices, then per local edge (a, b) the node next to a and the
// node next to b, then the faces (a, b, c) (2D: the interior node).  Edge
// nodes sit at (2 x_near + x_far) / 3, face nodes at ((x_p + x_q) + x_r) / 3
// with p < q < r the global vertex ids.  Interior vertices move by a
// seeded uniform jitter drawn from the SplitMix64 finaliser (Steele, Lea &
// Flood 2014) on the counter d*g + c; this file must be compiled without
// floating-point contraction so the coordinates are reproducible bit for bit.
#pragma once

#include <cstdint>
#include <vector>

namespace stokes {

// Incidence lists pack (simplex << kLocBits) | local index into an int32.
constexpr int kLocBits = 5;
constexpr int32_t kLocMask = (1 << kLocBits) - 1;

// `order` 2: Taylor-Hood P2/P1, 3: P3/P2.  The velocity space lives in
// p2 / n_p2 / p2coords / p2_bnd (P2 or P3 nodes), the pressure space in
// q / n_q / nqloc (the vertices, or the P2 nodes); vcoords / elems stay the
// vertex mesh that carries the geometry.
struct HostMesh {
  int dim = 0, n = 0, nloc = 0, order = 2, nqloc = 0;
  int64_t n_p1 = 0, n_p2 = 0, n_e = 0, n_q = 0;
  std::vector<double> vcoords;   // [n_p1][dim]
  std::vector<double> p2coords;  // [n_p2][dim] velocity node coordinates
  std::vector<int32_t> elems;    // [n_e][dim+1] vertex ids
  std::vector<int32_t> p2;       // [n_e][nloc] velocity node ids
  std::vector<uint8_t> p2_bnd;   // [n_p2] 1 on the boundary
  std::vector<int32_t> q;        // [n_e][nqloc] pressure node ids
};

struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;  // [nrows+1]
  std::vector<int32_t> cols;    // sorted within each row
};

// Problem-size arithmetic without building anything.
int64_t ipow(int64_t b, int e);

// Builds the mesh (order 2: P2/P1, 3: P3/P2); returns false if the sizes
// overflow 32-bit indices.
bool build_mesh(int dim, int n, uint64_t seed, double jitter, HostMesh& m, int order = 2);

// Pattern of (row_nodes[e][a], col_nodes[e][b]) pairs over all simplices.
// row_nodes has nr entries per simplex, col_nodes nc entries per simplex.
void element_pattern(const std::vector<int32_t>& row_nodes, int nr, int64_t nrows,
                     const std::vector<int32_t>& col_nodes, int nc, int64_t ncols, int64_t n_e,
                     HostCsr& out);

// Restrict rows and columns of a pattern through maps (-1 = dropped); the
// kept entries are renumbered and each row re-sorted.  src[k] receives the
// index of entry k in the input pattern.
void restrict_pattern(const HostCsr& in, const std::vector<int32_t>& row_map, int64_t nrows_out,
                      const std::vector<int32_t>& col_map, int64_t ncols_out, HostCsr& out,
                      std::vector<int64_t>* src);

// Transpose of a pattern; src[k] = index of the transposed entry in `in`.
void transpose_pattern(const HostCsr& in, HostCsr& out, std::vector<int64_t>& src);

// Pattern of A A^T through the middle index: row r of the output holds every
// row s of A that shares a kept column j (mid_keep[j] >= 0) with row r.
// At is the transpose pattern of A.  Rows come out sorted.
void product_pattern(const HostCsr& A, const HostCsr& At, const std::vector<int32_t>& mid_keep, HostCsr& out);

// Galerkin coarse operator P^T A P on the Kuhn hierarchy nf -> nc = nf / 2
// for the P1 interpolation that puts fine vertex f at the midpoint of the
// coarse edge (f - s, f + s) / 2, s = f mod 2 componentwise.  A is a P1 x P1
// operator on the (nf+1)^dim fine vertices; each output entry is summed in a
// fixed order.
void galerkin_p1(int dim, int nf, int nc, const HostCsr& A, const std::vector<double>& av, HostCsr& out,
                 std::vector<double>& ov);

// P2 interpolation from the Kuhn mesh with nf / 2 cells per side to the one
// with nf cells: row r is the fine P2 node fine_nat[r] (natural id on the
// (2 nf + 1)^dim grid), columns are the coarse interior P2 nodes (natural
// order among interior nodes of the (nf + 1)^dim grid), values the coarse
// P2 basis functions at the fine node of the unjittered nested meshes:
// lambda_a (2 lambda_a - 1) at vertices, 4 lambda_a lambda_b at edges.
// Coarse boundary nodes (Dirichlet) are dropped.
void p2_prolongation(int dim, int nf, const std::vector<int32_t>& fine_nat, HostCsr& P, std::vector<double>& pv);

// Incidence node -> (simplex << kLocBits | local index) for the node table
// nodes[e][0..nl), as CSR over n_nodes.
void incidence(const std::vector<int32_t>& nodes, int nl, int64_t n_e, int64_t n_nodes,
               std::vector<int64_t>& ptr, std::vector<int32_t>& list);

}  // namespace stokes

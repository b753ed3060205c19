// Host-side structured Kuhn mesh, P2/P1 numbering and sparsity patterns.
//
// The mesh is the unit square / cube cut into n^d cells, each split into d!
// simplices (Kuhn split): for every permutation pi of the axes, taken in
// lexicographic order, the simplex (v0, v0 + e_pi0, v0 + e_pi0 + e_pi1, ...,
// v0 + (1,..,1)).  P2 nodes are the points of the refined (2n+1)^d grid
// (vertex v -> 2v, edge (a, b) -> v_a + v_b).  Interior vertices move by a
// seeded uniform jitter drawn from the SplitMix64 finaliser (Steele, Lea &
// Flood 2014) on the counter d*g + c; this file must be compiled without
// floating-point contraction so the coordinates are reproducible bit for bit.
#pragma once

#include <cstdint>
#include <vector>

namespace stokes {

struct HostMesh {
  int dim = 0, n = 0, nloc = 0;
  int64_t n_p1 = 0, n_p2 = 0, n_e = 0;
  std::vector<double> vcoords;   // [n_p1][dim]
  std::vector<double> p2coords;  // [n_p2][dim]
  std::vector<int32_t> elems;    // [n_e][dim+1] vertex ids
  std::vector<int32_t> p2;       // [n_e][nloc] P2 node ids
  std::vector<uint8_t> p2_bnd;   // [n_p2] 1 on the boundary
};

struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;  // [nrows+1]
  std::vector<int32_t> cols;    // sorted within each row
};

// Problem-size arithmetic without building anything.
int64_t ipow(int64_t b, int e);

// Builds the mesh; returns false if the sizes overflow 32-bit indices.
bool build_mesh(int dim, int n, uint64_t seed, double jitter, HostMesh& m);

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

// Incidence node -> (simplex << 4 | local index) for the node table
// nodes[e][0..nl), as CSR over n_nodes.
void incidence(const std::vector<int32_t>& nodes, int nl, int64_t n_e, int64_t n_nodes,
               std::vector<int64_t>& ptr, std::vector<int32_t>& list);

}  // namespace stokes

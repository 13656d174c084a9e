// Host-side mesh tables for the uniform GLL spectral-element mesh of [0,L]^3.
// Paper: Sec. 2.4 (C0 Lagrange basis on GLL nodes, eq. fem; diagonal GLL mass;
// standard form eq. hep).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace chfsi {

struct MeshTables {
  double L = 0, h = 0;
  int n_el = 0, p = 0, q = 0;      // q = p + 1 nodes per direction
  int n = 0;                       // interior nodes per direction, n_el*p - 1
  int n_loc = 0;                   // q^3
  int np = 0;                      // n_loc rounded up to a multiple of 16 (MFMA tile)
  int64_t n_dof = 0, n_cells = 0;
  std::vector<double> xi, w;       // GLL nodes / weights on [-1,1]
  std::vector<double> D;           // D[qq*q + a] = l_a'(xi_qq)
  std::vector<double> K1;          // 1D reference stiffness, q x q
  std::vector<double> kcell;       // cell stiffness of -1/2 Laplacian, n_loc x n_loc
  std::vector<int32_t> cmap;       // [n_cells * n_loc], -1 = Dirichlet node
  std::vector<uint8_t> colors;     // [n_cells]
  std::vector<int32_t> cell_order; // cells sorted by colour
  int color_offset[9] = {0};
  std::vector<double> mass;        // [n_dof] diagonal of M
  double lam1d_max = 0;            // largest eigenvalue of the assembled 1D operator
  // periodic cell [0, L)^3: node index I = (ex p + a) mod (n_el p), n = n_el p,
  // no Dirichlet nodes; gcell[d] = int N_j d_d N_l (GLL rule), n_loc x n_loc
  bool periodic = false;
  std::vector<double> gcell[3];
};

// Builds every table; returns an empty string on success, else a message.
// periodic: the Bloch-periodic cell of Sec. 2.1 (n_el even, so that the
// 8-colour parity rule still separates cells that share a node across the wrap).
std::string build_mesh(double L, int n_el, int p, MeshTables &m, bool periodic = false);

// Largest eigenvalue (or, above 200 nodes, a Gershgorin bound of it) of the
// 1D Bloch operator m^-1/2 (1/2 K1D - i k C1D + 1/2 k^2 m) m^-1/2 on the
// n_el p periodic nodes of a periodic mesh; the sum over the three directions
// plus max V bounds lambda_max(Htilde_k) (Weyl, Kronecker sum).
double bloch_1d_max(const MeshTables &m, double k);

// x,y,z of every interior node in dof order.
void dof_coords(const MeshTables &m, double *xyz);

// GLL rule of degree p (p+1 nodes ascending, weights).
void gll_rule(int p, std::vector<double> &xi, std::vector<double> &w);

// Eigenvalues of a dense symmetric matrix (cyclic Jacobi, host, small n).
void sym_eigvals(std::vector<double> a, int n, std::vector<double> &out);

}  // namespace chfsi

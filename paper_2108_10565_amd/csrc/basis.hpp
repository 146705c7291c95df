// Host construction of the predictor's reference matrices (float64).
//
// Spatial: Dubiner basis on the reference tetrahedron (subsection "Spatial
// discretisation" of Wolf et al., arXiv 2108.10565), mass matrix
// M_kl = int phi_k phi_l and stiffness matrices K^a_kl = int phi_k d_a phi_l
// (definitions after eq:stp), by Gauss-Legendre quadrature in collapsed
// coordinates with analytic derivatives of the Jacobi factors;
// Khat^a = M^-1 K^a (section "Block-wise back-substitution").
// Temporal: Legendre basis on [0, 1]; Z = S^-1 (W - K^tau) and S^-1 w.
#pragma once

#include <vector>

namespace stp_host {

constexpr int kNQ = 13;
constexpr int kMaxDegree = 7;

constexpr int n_modes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
constexpr int block_size(int g) { return (g + 1) * (g + 2) / 2; }
constexpr int block_start(int g) { return g * (g + 1) * (g + 2) / 6; }

struct ReferenceMatrices {
  int N = -1;
  int B = 0, T = 0;
  std::vector<double> Z;      // [T][T]
  std::vector<double> Sinv_w; // [T]
  std::vector<double> M;      // [B]  (diagonal of the mass matrix)
  std::vector<double> K;      // [3][B][B]
  std::vector<double> Khat;   // [3][B][B]
  double max_mass_offdiag = 0;  // quadrature check: should be ~1e-17
};

// (i, j, k) of spatial mode m in the ABI order.
void mode_ijk(int N, int m, int* i, int* j, int* k);

// Builds every matrix above for degree N (0..kMaxDegree).
ReferenceMatrices build_reference_matrices(int N);

}  // namespace stp_host

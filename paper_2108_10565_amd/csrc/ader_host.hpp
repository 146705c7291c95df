// Host side of the ADER-DG corrector: reference tables, the Dubiner basis at
// points, the upwind split of a normal Jacobian and per-face flux operators.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "basis.hpp"

namespace stp_host {

// Local vertex triples of the faces of the reference tetrahedron
// (vertices (0,0,0), (1,0,0), (0,1,0), (0,0,1)); face f is parameterised by
// x = V[a] + s (V[b] - V[a]) + t (V[c] - V[a]), s, t >= 0, s + t <= 1.
constexpr int kFaceVertices[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};

// phi[0..B) = the Dubiner basis of degree N (ABI order) at (x, y, z).
void eval_dubiner(int N, double x, double y, double z, double* phi);

// Reference tables of the corrector, all divided by the mass M_kk of the
// test function k (the left-hand side of eq:semi_discrete):
//   V  [3][B][B]      V^d_lk = int phi_l d_d phi_k / M_kk       (volume)
//   Fl [4][B][B]      int_face_i phi_l phi_k ds dt / M_kk       (own face)
//   Fn [4][4][6][B][B] int_face_i phi_l(neighbour face j under vertex
//                      correspondence h) phi_k ds dt / M_kk     (neighbour)
// Correspondence h: the own face's vertex r is the neighbour face's vertex
// kPerm[h][r], kPerm = {012, 021, 102, 120, 201, 210}.
struct CorrectorTables {
  int N = -1, B = 0;
  std::vector<double> M, V, Fl, Fn;
};
CorrectorTables build_corrector_tables(int N);

// Godunov split of a normal Jacobian An (nq x nq, real spectrum,
// diagonalisable): An^+ = R max(Lambda, 0) R^-1, An^- = An - An^+.
// Eigenvalues by balanced Hessenberg QR; the split by spectral projectors.
bool upwind_split(int nq, const double* An, double* Ap, double* Am, std::string* err);

// Per element e and face f of a mesh (verts [n][4][3], physical Jacobians
// ABC [n][3][nq][nq]): with the outward unit normal nu and the area |S| of
// the face and |J| = |det| of the element map,
//   Gp[e][f] = (2 |S| / |J|) An^+,  Gm[e][f] = (2 |S| / |J|) An^-,
// An = nu_x A + nu_y B + nu_z C.
bool face_operators(int nq, int64_t n, const double* ABC, const double* verts, double* Gp, double* Gm,
                    std::string* err);

}  // namespace stp_host

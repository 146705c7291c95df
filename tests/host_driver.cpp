// Host-only driver for the sanitizer test: runs the library's host code
// (reference matrices and their quadrature, the Dubiner basis, corrector
// tables, Godunov upwind split and face operators) on inputs read from a
// file, and writes the results for comparison with the library build.
//
//   host_driver IN OUT
//   IN : int32 nq, int32 degree, int64 n, ABC [n][3][nq][nq] f64,
//        verts [n][4][3] f64
//   OUT: Khat [3][B][B], corrector tables (M, V, Fl, Fn), phi at 7 points
//        [7][B], Gp [n][4][nq][nq], Gm [n][4][nq][nq] (all f64)
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../paper_2108_10565_amd/csrc/ader_host.hpp"
#include "../paper_2108_10565_amd/csrc/basis.hpp"

namespace {

bool read_all(std::FILE* f, void* p, size_t bytes) { return std::fread(p, 1, bytes, f) == bytes; }

void write_vec(std::FILE* f, const std::vector<double>& v) { std::fwrite(v.data(), sizeof(double), v.size(), f); }

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: host_driver IN OUT\n");
    return 2;
  }
  std::FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 3;
  int32_t nq = 0, degree = 0;
  int64_t n = 0;
  if (!read_all(in, &nq, 4) || !read_all(in, &degree, 4) || !read_all(in, &n, 8)) return 4;
  std::vector<double> ABC(static_cast<size_t>(n) * 3 * nq * nq), verts(static_cast<size_t>(n) * 12);
  if (!read_all(in, ABC.data(), ABC.size() * 8) || !read_all(in, verts.data(), verts.size() * 8)) return 5;
  std::fclose(in);

  // every degree's reference matrices (the quadrature and the Khat products)
  stp_host::ReferenceMatrices R;
  for (int N = 0; N <= stp_host::kMaxDegree; ++N) {
    const stp_host::ReferenceMatrices r = stp_host::build_reference_matrices(N);
    if (r.max_mass_offdiag > 1e-12) {
      std::fprintf(stderr, "mass matrix not diagonal at N=%d\n", N);
      return 6;
    }
    if (N == degree) R = r;
  }
  const stp_host::CorrectorTables C = stp_host::build_corrector_tables(degree);
  const double pts[7][3] = {{0.25, 0.25, 0.25}, {0.0, 0.0, 0.0}, {1.0, 0.0, 0.0}, {0.0, 1.0, 0.0},
                            {0.0, 0.0, 1.0},    {0.1, 0.2, 0.3}, {0.5, 0.5, 0.0}};
  std::vector<double> phi(7 * static_cast<size_t>(R.B));
  for (int i = 0; i < 7; ++i) stp_host::eval_dubiner(degree, pts[i][0], pts[i][1], pts[i][2], &phi[i * R.B]);
  std::vector<double> Gp(static_cast<size_t>(n) * 4 * nq * nq), Gm(Gp.size());
  std::string err;
  if (!stp_host::face_operators(nq, n, ABC.data(), verts.data(), Gp.data(), Gm.data(), &err)) {
    std::fprintf(stderr, "face_operators: %s\n", err.c_str());
    return 7;
  }
  std::FILE* out = std::fopen(argv[2], "wb");
  if (!out) return 8;
  write_vec(out, R.Khat);
  write_vec(out, C.M);
  write_vec(out, C.V);
  write_vec(out, C.Fl);
  write_vec(out, C.Fn);
  write_vec(out, phi);
  write_vec(out, Gp);
  write_vec(out, Gm);
  std::fclose(out);
  return 0;
}

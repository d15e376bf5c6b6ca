// Test driver (CPU only): runs the library's host set-up of triangle meshes
// and the triangle oracle under AddressSanitizer and UndefinedBehavior-
// Sanitizer.  Built and run by tests/test_sanitizers.py on seeded meshes it
// writes to a scratch directory:  san2d <dir> <tag>...  where <dir>/<tag>.txt
// holds "n_vert n_cell px py" and <tag>.xy, <tag>.tri, <tag>.u the arrays.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "../../paper_2105_02127_amd/csrc/internal.h"
#include "../../oracle/teno_oracle.cpp"

namespace teno {
const char* last_error();
}

template <class T>
static std::vector<T> slurp(const std::string& path, size_t n) {
  std::vector<T> v(n);
  std::ifstream f(path, std::ios::binary);
  f.read(reinterpret_cast<char*>(v.data()), (std::streamsize)(n * sizeof(T)));
  if (!f) {
    std::fprintf(stderr, "cannot read %s\n", path.c_str());
    std::exit(2);
  }
  return v;
}

static void check(bool ok, const char* what, const std::string& tag) {
  if (!ok) {
    std::fprintf(stderr, "FAILED %s on %s: %s / %s\n", what, tag.c_str(), teno::last_error(),
                 oracle_last_error());
    std::exit(3);
  }
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string dir = argv[1];
  oracle_set_threads(1);
  for (int t = 2; t < argc; ++t) {
    const std::string tag = argv[t];
    int nv = 0, nc = 0;
    double per[2] = {0, 0};
    {
      std::ifstream h(dir + "/" + tag + ".txt");
      h >> nv >> nc >> per[0] >> per[1];
    }
    const auto xy = slurp<double>(dir + "/" + tag + ".xy", 2 * (size_t)nv);
    const auto tri = slurp<int32_t>(dir + "/" + tag + ".tri", 3 * (size_t)nc);
    const auto U = slurp<double>(dir + "/" + tag + ".u", 4 * (size_t)nc);
    const bool open = !(per[0] > 0 && per[1] > 0);
    // ---- library set-up: every order, conservative and characteristic ----
    for (int order = 3; order <= 6; ++order)
      for (int ch = 0; ch <= 1; ++ch) {
        teno::Mesh m;
        check(teno::mesh_create(nv, xy.data(), nc, tri.data(), per, m) == 0, "mesh_create", tag);
        if (open) {
          m.bkind.assign(m.bface.size(), 0);
          for (size_t b = 0; b < m.bface.size(); ++b) m.bkind[b] = 1 + (int)(b % 2);
        }
        teno_params p{};
        p.order = order;
        p.power = 6;
        p.ct = 1e-6;
        p.eps = 1e-12;
        p.gamma = 1.4;
        p.tie_rel = 1e-10;
        p.fallback = 1;
        p.reorder = 1;
        p.n_threads = 2;
        p.characteristic = ch;
        p.dk_prime = 1e4;
        check(teno::mesh_setup(m, p) == 0, "mesh_setup", tag);
        double s = 0.0;
        for (int i = 0; i < nc; i += 7)
          for (int k = 0; k < 4; ++k) {
            const int nrow = k == 3 ? m.d.nl : teno::kSmallRows;
            const int nco = k == 3 ? m.d.nu : teno::kSmallCoef;
            for (int r = 0; r < nrow; ++r)
              for (int l = 0; l < nco; ++l) s += m.M[teno::packed_M_offset(m.d, m.inv[i], k, r, l)];
          }
        check(s == s, "operator readback", tag);
      }
    // ---- oracle: residual, RK step, adjoint ----
    for (int order = 3; order <= 6; order += 3) {
      void* h = oracle_mesh_create(nv, xy.data(), nc, tri.data(), per);
      check(h != nullptr, "oracle_mesh_create", tag);
      if (open) {
        const int nb = oracle_boundary_count(h);
        std::vector<int> kind(nb);
        std::vector<double> st(4 * (size_t)nb);
        for (int b = 0; b < nb; ++b) {
          kind[b] = 1 + b % 3;
          st[4 * b] = 1.0;
          st[4 * b + 1] = 0.1;
          st[4 * b + 2] = 0.0;
          st[4 * b + 3] = 2.5;
        }
        check(oracle_set_boundary(h, kind.data(), st.data()) == 0, "oracle_set_boundary", tag);
      }
      oracle_params op;
      oracle_default_params(&op);
      op.order = order;
      op.fallback = 1;
      check(oracle_setup(h, &op, 1) == 0, "oracle_setup", tag);
      std::vector<double> R(4 * (size_t)nc), U1(4 * (size_t)nc), st(12 * (size_t)nc), Ub(4 * (size_t)nc);
      std::vector<uint16_t> fl(nc), fl3(3 * (size_t)nc), ties(nc), ties3(3 * (size_t)nc);
      oracle_diag dg{};
      check(oracle_residual(h, U.data(), R.data(), fl.data(), 0, nullptr, &dg, ties.data()) == 0,
            "oracle_residual", tag);
      const double dt = oracle_dt(h, U.data(), 0.4);
      check(dt > 0.0, "oracle_dt", tag);
      check(oracle_rk_step(h, U.data(), U1.data(), dt, fl3.data(), 0, st.data(), &dg, ties3.data()) == 0,
            "oracle_rk_step", tag);
      check(oracle_vjp(h, U.data(), fl.data(), R.data(), Ub.data()) == 0, "oracle_vjp", tag);
      oracle_mesh_destroy(h);
    }
    std::printf("%s ok\n", tag.c_str());
  }
  return 0;
}

// Test driver (CPU only): runs the library's host set-up of tetrahedral
// meshes and the tetrahedral oracle under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Built and run by tests/test_sanitizers.py:
// san3d <dir> <tag>...  where <dir>/<tag>.txt holds "n_vert n_cell px py pz"
// and <tag>.xyz, <tag>.tet, <tag>.u the arrays.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "../../paper_2105_02127_amd/csrc/internal3.h"
#include "../../oracle/teno3_oracle.cpp"

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
                 oracle3_last_error());
    std::exit(3);
  }
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string dir = argv[1];
  oracle3_set_threads(1);
  for (int t = 2; t < argc; ++t) {
    const std::string tag = argv[t];
    int nv = 0, nc = 0;
    double per[3] = {0, 0, 0};
    {
      std::ifstream h(dir + "/" + tag + ".txt");
      h >> nv >> nc >> per[0] >> per[1] >> per[2];
    }
    const auto xyz = slurp<double>(dir + "/" + tag + ".xyz", 3 * (size_t)nv);
    const auto tet = slurp<int32_t>(dir + "/" + tag + ".tet", 4 * (size_t)nc);
    const auto U = slurp<double>(dir + "/" + tag + ".u", 5 * (size_t)nc);
    const bool open = !(per[0] > 0 && per[1] > 0 && per[2] > 0);
    // ---- library set-up, orders 3 and 4 ----
    for (int order = 3; order <= 4; ++order) {
      teno::Mesh3 m;
      check(teno::mesh3_create(nv, xyz.data(), nc, tet.data(), per, m) == 0, "mesh3_create", tag);
      if (open)
        for (size_t b = 0; b < m.bkind.size(); ++b) m.bkind[b] = 1 + (int)(b % 2);
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
      check(teno::mesh3_setup(m, p) == 0, "mesh3_setup", tag);
      double s = 0.0;
      for (double x : m.M) s += x;
      check(s == s, "operators", tag);
    }
    // ---- oracle: residual, dt, RK step ----
    void* h = oracle3_mesh_create(nv, xyz.data(), nc, tet.data(), per);
    check(h != nullptr, "oracle3_mesh_create", tag);
    int onc = 0, onf = 0, onb = 0;
    oracle3_mesh_counts(h, &onc, &onf, &onb);
    if (onb > 0) {
      std::vector<int> kind(onb);
      for (int b = 0; b < onb; ++b) kind[b] = 1 + b % 2;
      check(oracle3_set_boundary(h, kind.data()) == 0, "oracle3_set_boundary", tag);
    }
    oracle3_params op{};
    op.order = 3;
    op.power = 6;
    op.fallback = 1;
    op.ct = 1e-6;
    op.eps = 1e-12;
    op.gamma = 1.4;
    op.tie_rel = 1e-10;
    check(oracle3_setup(h, &op, 1) == 0, "oracle3_setup", tag);
    std::vector<double> R(5 * (size_t)nc), U1(5 * (size_t)nc), st(15 * (size_t)nc);
    std::vector<uint32_t> fl(nc), fl3(3 * (size_t)nc), ties(nc), ties3(3 * (size_t)nc);
    oracle3_diag dg{};
    check(oracle3_residual(h, U.data(), R.data(), fl.data(), 0, nullptr, &dg, ties.data()) == 0,
          "oracle3_residual", tag);
    const double dt = oracle3_dt(h, U.data(), 0.4);
    check(dt > 0.0, "oracle3_dt", tag);
    check(oracle3_rk_step(h, U.data(), U1.data(), dt, fl3.data(), 0, st.data(), &dg, ties3.data()) == 0,
          "oracle3_rk_step", tag);
    oracle3_mesh_destroy(h);
    std::printf("%s ok\n", tag.c_str());
  }
  return 0;
}

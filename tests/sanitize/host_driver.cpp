// host_driver.cpp -- exercises libmdg's host setup (setup.cpp: mesh
// canonicalisation, face matching, geometry records, element ordering,
// tiles, halo codes, PML and dipole records, projection and state packing)
// in a host-only build with AddressSanitizer and UndefinedBehaviorSanitizer.
// Checks structural invariants along the way; any sanitizer report or failed
// check ends the program with a non-zero status. Test infrastructure only.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "refbasis.hpp"
#include "solver.hpp"

using namespace mdg;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(3);                                                 \
    }                                                               \
  } while (0)

// n^3 cubes of [0,1]^3 split into 6 tetrahedra each (monotone lattice paths)
static void kuhn(int n, std::vector<double>& xyz, std::vector<int64_t>& tet, std::mt19937& rng, double jit) {
  const int m = n + 1;
  xyz.assign(size_t(m) * m * m * 3, 0.0);
  std::uniform_real_distribution<double> u(-jit, jit);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        double* p = &xyz[((size_t(k) * m + j) * m + i) * 3];
        const bool inner = i > 0 && j > 0 && k > 0 && i < n && j < n && k < n;
        p[0] = (i + (inner ? u(rng) : 0.0)) / n;
        p[1] = (j + (inner ? u(rng) : 0.0)) / n;
        p[2] = (k + (inner ? u(rng) : 0.0)) / n;
      }
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  tet.clear();
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (auto& pr : perms) {
          int c[3] = {i, j, k};
          int64_t v[4];
          v[0] = (int64_t(c[2]) * m + c[1]) * m + c[0];
          for (int s = 0; s < 3; ++s) {
            c[pr[s]] += 1;
            v[s + 1] = (int64_t(c[2]) * m + c[1]) * m + c[0];
          }
          // a random vertex order inside the tet: the library sorts it
          std::shuffle(v, v + 4, rng);
          tet.insert(tet.end(), v, v + 4);
        }
}

static void init(Solver& s, int order, int precision, int flux, int mixed, double sip) {
  s = Solver();
  s.opt.order = order;
  s.opt.precision = precision;
  s.opt.flux = flux;
  s.opt.integrator = MDG_RK4;
  s.opt.cfl = 0.3;
  s.opt.mixed = mixed;
  s.opt.sip_alpha = sip;
  s.P = order + mixed;
  s.N = nmodes3(s.P);
  s.NF = nmodes2(s.P);
  s.NH = nmodes3(order);
  s.NFH = nmodes2(order);
}

static void check_decomposition(const Solver& s) {
  CHECK(s.finalized);
  CHECK(s.K == s.nt && s.Kpad % 64 == 0 && s.Kpad >= s.K);
  std::vector<int> seen(s.nt, 0);
  for (int64_t k = 0; k < s.K; ++k) {
    CHECK(s.perm[k] >= 0 && s.perm[k] < s.nt);
    CHECK(s.iperm[s.perm[k]] == k);
    seen[s.perm[k]]++;
  }
  for (int c : seen) CHECK(c == 1);
  int64_t halo = 0;
  for (int64_t k = 0; k < s.K; ++k)
    for (int f = 0; f < 4; ++f) {
      const int32_t g = s.nbr_glob[size_t(k) * 4 + f];
      if (g >= 0) {
        CHECK(g / 4 < s.K);
        CHECK(s.nbr_glob[size_t(g / 4) * 4 + g % 4] == int32_t(k * 4 + f));  // symmetric
      }
      const int32_t pc = s.pub_code[blk_index(k, f, 4)];
      if (pc >= 0) {
        ++halo;
        CHECK(int64_t(pc) + halo_role_reals(s.NF, int(s.real_size())) <= s.hreg);
      }
    }
  CHECK(halo == s.nhalo);
  for (int64_t t = 0; t < s.ntiles; ++t) CHECK(s.halo_tile[2 * t + 1] >= 0 && s.halo_tile[2 * t + 1] <= s.hmax);
  CHECK(s.L.total > 0 && s.L.total % 256 == 0);
}

static void roundtrip(const Solver& s, std::mt19937& rng) {
  std::normal_distribution<double> g;
  std::vector<double> E(size_t(s.nt) * 3 * s.N), H(size_t(s.nt) * 3 * s.NH), E2(E.size()), H2(H.size()), buf;
  for (auto& x : E) x = g(rng);
  for (auto& x : H) x = g(rng);
  pack_state(s, E.data(), H.data(), buf);
  unpack_state(s, buf, E2.data(), H2.data());
  CHECK(E == E2 && H == H2);
  if (s.Kp > 0) {
    std::vector<double> P(E.size()), Q(H.size()), P2(E.size()), Q2(H.size());
    for (auto& x : P) x = g(rng);
    for (auto& x : Q) x = g(rng);
    pack_aux(s, P.data(), Q.data(), buf);
    unpack_aux(s, buf, P2.data(), Q2.data());
    for (int64_t k = 0; k < s.nt; ++k) {
      const bool damped = s.omega[size_t(k) * 3] > 0 || s.omega[size_t(k) * 3 + 1] > 0 || s.omega[size_t(k) * 3 + 2] > 0;
      for (int i = 0; i < 3 * s.N && damped; ++i)
        CHECK(std::fabs(P2[size_t(k) * 3 * s.N + i] - P[size_t(k) * 3 * s.N + i]) < 1e-9 * (1 + std::fabs(P[size_t(k) * 3 * s.N + i])));
    }
  }
  if (s.sip()) {
    std::vector<double> S(size_t(s.nt) * 8 * s.NFH), S2(S.size());
    for (auto& x : S) x = g(rng);
    pack_sip(s, S.data(), buf);
    unpack_sip(s, buf, S2.data());
    CHECK(S == S2);
  }
  const int q = 3;
  std::vector<double> x(size_t(s.nt) * q * q * q * 3), coef;
  projection_points(s, q, x.data());
  project_fields(s, q, x.data(), s.N, coef);  // the field (x, y, z) itself
  CHECK(coef.size() == size_t(s.nt) * 3 * s.N);
  for (double c : coef) CHECK(std::isfinite(c));
}

static int expect_error(Solver& s, std::vector<double> xyz, std::vector<int64_t> tet) {
  try {
    setup_mesh(s, int64_t(xyz.size() / 3), xyz.data(), int64_t(tet.size() / 4), tet.data());
  } catch (const Error& e) {
    return e.code;
  }
  return 0;
}

int main() {
  std::mt19937 rng(7);
  int cases = 0;
  for (int n : {1, 2, 5}) {
    for (int prec : {MDG_FP64, MDG_FP32}) {
      for (int variant = 0; variant < 4; ++variant) {
        std::vector<double> xyz;
        std::vector<int64_t> tet;
        kuhn(n, xyz, tet, rng, n > 1 ? 0.1 : 0.0);
        const int64_t nt = int64_t(tet.size() / 4);
        Solver s;
        const int flux = variant == 1 ? MDG_UPWIND : MDG_CENTRAL;
        init(s, variant == 2 ? 2 : 3, prec, flux, variant == 2 ? 1 : 0, variant == 3 ? 1.0 : 0.0);
        setup_mesh(s, int64_t(xyz.size() / 3), xyz.data(), nt, tet.data());
        std::vector<double> eps(nt), mu(nt), omega(size_t(nt) * 3, 0.0);
        std::uniform_real_distribution<double> u(1.0, 4.0);
        for (auto& e : eps) e = u(rng);
        for (auto& m : mu) m = 1.0 + 0.5 * (u(rng) - 1.0);
        setup_material(s, eps.data(), mu.data());
        if (variant != 3) {  // PML on a third of the elements, one axis undamped on some
          for (int64_t k = 0; k < nt; k += 3) {
            omega[size_t(k) * 3] = 2.0;
            omega[size_t(k) * 3 + 1] = (k % 2) ? 0.0 : 1.5;
            omega[size_t(k) * 3 + 2] = 3.0;
          }
          setup_pml(s, omega.data());
        }
        const double pos[6] = {0.41, 0.52, 0.47, 0.2, 0.3, 0.6}, dir[6] = {0, 0, 1, 1, 0, 0};
        const double wave[6] = {2.0, 1.0, 0.8, 1.0, 2.0, 0.5};
        setup_dipoles(s, 2, nullptr, pos, dir, wave);
        finalize(s);
        check_decomposition(s);
        CHECK(cfl_dt(s) > 0);
        CHECK(bytes_per_stage(s) > 0 && flops_per_stage(s) > 0);
        roundtrip(s, rng);
        ++cases;
      }
    }
  }
  // instances: two meshes side by side
  {
    std::vector<double> a, b;
    std::vector<int64_t> ta, tb;
    kuhn(2, a, ta, rng, 0.1);
    kuhn(3, b, tb, rng, 0.1);
    const int64_t nva = int64_t(a.size() / 3);
    for (size_t i = 0; i < b.size(); i += 3) b[i] += 2.0;
    a.insert(a.end(), b.begin(), b.end());
    for (auto v : tb) ta.push_back(v + nva);
    Solver s;
    init(s, 3, MDG_FP32, MDG_UPWIND, 0, 0.0);
    setup_mesh(s, int64_t(a.size() / 3), a.data(), int64_t(ta.size() / 4), ta.data());
    const int64_t bounds[3] = {0, 48, 48 + 162};  // 2^3 and 3^3 cubes x 6
    setup_instances(s, 2, bounds);
    finalize(s);
    check_decomposition(s);
    roundtrip(s, rng);
    ++cases;
  }
  // error paths
  {
    std::vector<double> xyz;
    std::vector<int64_t> tet;
    kuhn(1, xyz, tet, rng, 0.0);
    Solver s;
    init(s, 2, MDG_FP64, MDG_CENTRAL, 0, 0.0);
    std::vector<int64_t> bad = tet;
    bad[1] = bad[0];
    CHECK(expect_error(s, xyz, bad) == MDG_E_MESH);
    bad = tet;
    bad[3] = 99;
    CHECK(expect_error(s, xyz, bad) == MDG_E_ARG);
    std::vector<double> flat = xyz;
    for (size_t i = 2; i < flat.size(); i += 3) flat[i] = 0.0;
    CHECK(expect_error(s, flat, tet) == MDG_E_MESH);
    std::vector<double> nanv = xyz;
    nanv[4] = NAN;
    CHECK(expect_error(s, nanv, tet) == MDG_E_MESH);
    ++cases;
  }
  std::printf("host setup: %d cases clean\n", cases);
  return 0;
}

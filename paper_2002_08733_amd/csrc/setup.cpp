// setup.cpp -- host-side setup of libmdg: mesh canonicalisation, face
// matching, element geometry, element ordering and tiling for the stage
// kernel, PML and source records, projection and state (un)packing.
//
// Geometry [KS Sec. II]: every tetrahedron is stored with its vertices sorted
// by ascending global id; A = [v1-v0, v2-v0, v3-v0] (eq. mapping_template).
// With the covariant basis A^-T e_j phi_l (eq. mapped_eh):
//   mass     (eps phi_jl, phi_km)_T = eps |det A| (A^-1 A^-T)_jk delta_lm      [KS Sec. III]
//   curl     (curl phi_jl, phi_km)_T = sign(det A) (curl^ phi^_jl, phi^_km)_T^ [eq. matrix_free_curl]
// so the only per-element data of the operator are G0^-1 = A^T A / |det A|,
// sign(det A), 1/eps, 1/mu (and impedance weights for the upwind flux).
//
// Face coupling: a face is parametrised from its three vertices in ascending
// global-id order on both of its elements, so both elements see the same
// physical point at the same parameter s and the same tangents t1, t2; their
// face-basis coefficients can be combined without any permutation.
#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <utility>

#include "refbasis.hpp"
#include "refops_gen.h"
#include "solver.hpp"

namespace mdg {

static void inv3(const double* a, double* r, double* det_out) {
  const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
  *det_out = det;
  const double id = 1.0 / det;
  r[0] = (a[4] * a[8] - a[5] * a[7]) * id;
  r[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  r[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  r[3] = (a[5] * a[6] - a[3] * a[8]) * id;
  r[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  r[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  r[6] = (a[3] * a[7] - a[4] * a[6]) * id;
  r[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  r[8] = (a[0] * a[4] - a[1] * a[3]) * id;
}

void setup_mesh(Solver& s, int64_t nv, const double* xyz, int64_t nt, const int64_t* tet) {
  if (nv < 4 || nt < 1 || !xyz || !tet) throw Error(MDG_E_ARG, "set_mesh: empty mesh or NULL array");
  for (int64_t i = 0; i < 3 * nv; ++i)
    if (!std::isfinite(xyz[i])) throw Error(MDG_E_MESH, "set_mesh: non-finite vertex coordinate");
  s.nv = nv;
  s.nt = nt;
  s.xyz.assign(xyz, xyz + 3 * nv);
  s.tet.resize(4 * nt);
  for (int64_t k = 0; k < nt; ++k) {
    int64_t* t = &s.tet[4 * k];
    for (int v = 0; v < 4; ++v) {
      t[v] = tet[4 * k + v];
      if (t[v] < 0 || t[v] >= nv) throw Error(MDG_E_ARG, "set_mesh: vertex id out of range in tet " + std::to_string(k));
    }
    std::sort(t, t + 4);
    for (int v = 0; v < 3; ++v)
      if (t[v] == t[v + 1]) throw Error(MDG_E_MESH, "set_mesh: repeated vertex in tet " + std::to_string(k));
  }
  // geometry
  s.A.resize(9 * nt);
  s.Ainv.resize(9 * nt);
  s.det.resize(nt);
  for (int64_t k = 0; k < nt; ++k) {
    const double* x0 = &s.xyz[3 * s.tet[4 * k]];
    double* A = &s.A[9 * k];
    double emax = 0;
    for (int c = 0; c < 3; ++c) {
      const double* xc = &s.xyz[3 * s.tet[4 * k + c + 1]];
      for (int r = 0; r < 3; ++r) {
        A[3 * r + c] = xc[r] - x0[r];
        emax = std::max(emax, std::fabs(A[3 * r + c]));
      }
    }
    double det;
    inv3(A, &s.Ainv[9 * k], &det);
    if (!std::isfinite(det) || std::fabs(det) <= 1e-12 * emax * emax * emax)
      throw Error(MDG_E_MESH, "set_mesh: degenerate (zero-volume) tet " + std::to_string(k));
    s.det[k] = det;
  }
  // faces: sort face-sides by their vertex triple and pair equal neighbours
  struct FS { int64_t a, b, c, side; };
  std::vector<FS> fs(4 * nt);
  for (int64_t k = 0; k < nt; ++k)
    for (int f = 0; f < 4; ++f) {
      int fv[3];
      face_vertices(f, fv);
      const int64_t* t = &s.tet[4 * k];
      fs[4 * k + f] = {t[fv[0]], t[fv[1]], t[fv[2]], 4 * k + f};
    }
  std::sort(fs.begin(), fs.end(), [](const FS& x, const FS& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.side < y.side;
  });
  s.side.assign(4 * nt, -1);
  s.n_int = s.n_bnd = 0;
  for (size_t i = 0; i < fs.size();) {
    size_t j = i + 1;
    while (j < fs.size() && fs[j].a == fs[i].a && fs[j].b == fs[i].b && fs[j].c == fs[i].c) ++j;
    if (j - i > 2) throw Error(MDG_E_MESH, "set_mesh: face shared by more than two tets");
    if (j - i == 2) {
      s.side[fs[i].side] = fs[i + 1].side;
      s.side[fs[i + 1].side] = fs[i].side;
      ++s.n_int;
    } else {
      ++s.n_bnd;
    }
    i = j;
  }
  s.eps.assign(nt, 1.0);
  s.mu.assign(nt, 1.0);
  s.omega.clear();
  s.dips.clear();
  s.inst_first = {0, nt};
  s.inst_of.assign(nt, 0);
  s.finalized = false;
  s.bound = false;
  s.t0 = 0.0;
  s.nstep = 0;
}

void setup_material(Solver& s, const double* eps, const double* mu) {
  for (int64_t k = 0; k < s.nt; ++k) {
    const double e = eps ? eps[k] : 1.0, m = mu ? mu[k] : 1.0;
    if (!(e > 0) || !(m > 0) || !std::isfinite(e) || !std::isfinite(m))
      throw Error(MDG_E_ARG, "set_material: eps and mu must be positive and finite");
  }
  s.eps.assign(s.nt, 1.0);
  s.mu.assign(s.nt, 1.0);
  if (eps) std::copy(eps, eps + s.nt, s.eps.begin());
  if (mu) std::copy(mu, mu + s.nt, s.mu.begin());
  s.finalized = false;
  s.bound = false;
}

void setup_pml(Solver& s, const double* omega) {
  if (!omega) {
    s.omega.clear();
  } else {
    for (int64_t i = 0; i < 3 * s.nt; ++i)
      if (!(omega[i] >= 0) || !std::isfinite(omega[i]))
        throw Error(MDG_E_ARG, "set_pml: damping must be finite and >= 0");
    s.omega.assign(omega, omega + 3 * s.nt);
  }
  s.finalized = false;
  s.bound = false;
}

void setup_instances(Solver& s, int n, const int64_t* first) {
  if (n < 1 || !first) throw Error(MDG_E_ARG, "set_instances: n >= 1 and first[n+1] required");
  if (first[0] != 0 || first[n] != s.nt) throw Error(MDG_E_ARG, "set_instances: first[0] = 0 and first[n] = nt");
  for (int i = 0; i < n; ++i)
    if (first[i + 1] <= first[i]) throw Error(MDG_E_ARG, "set_instances: empty or decreasing range");
  std::vector<int32_t> of(s.nt);
  for (int i = 0; i < n; ++i)
    for (int64_t k = first[i]; k < first[i + 1]; ++k) of[k] = i;
  for (int64_t k = 0; k < s.nt; ++k)
    for (int f = 0; f < 4; ++f) {
      const int64_t sd = s.side[4 * k + f];
      if (sd >= 0 && of[sd / 4] != of[k])
        throw Error(MDG_E_MESH, "set_instances: a face joins instances " + std::to_string(of[k]) + " and " +
                                    std::to_string(of[sd / 4]));
    }
  s.inst_first.assign(first, first + n + 1);
  s.inst_of.swap(of);
  s.dips.clear();
  s.finalized = false;
  s.bound = false;
}

void setup_dipoles(Solver& s, int n, const int32_t* inst, const double* pos, const double* dir,
                   const double* wave) {
  if (n < 0) throw Error(MDG_E_ARG, "set_dipoles: n >= 0");
  if (n > 0 && (!pos || !dir || !wave)) throw Error(MDG_E_ARG, "set_dipoles: NULL array");
  const int ninst = (int)s.inst_first.size() - 1;
  std::vector<Dipole> out;
  std::vector<double> val(s.N);
  for (int d = 0; d < n; ++d) {
    Dipole dp;
    for (int c = 0; c < 3; ++c) {
      dp.pos[c] = pos[3 * d + c];
      dp.dir[c] = dir[3 * d + c];
      dp.wave[c] = wave[3 * d + c];
    }
    if (!(dp.wave[1] > 0)) throw Error(MDG_E_ARG, "set_dipoles: bandwidth must be > 0");
    dp.inst = inst ? inst[d] : -1;
    if (dp.inst < -1 || dp.inst >= ninst) throw Error(MDG_E_ARG, "set_dipoles: instance out of range");
    const int64_t k0 = dp.inst < 0 ? 0 : s.inst_first[dp.inst];
    const int64_t k1 = dp.inst < 0 ? s.nt : s.inst_first[dp.inst + 1];
    dp.elem = -1;
    double rh[3] = {0, 0, 0};
    for (int64_t k = k0; k < k1 && dp.elem < 0; ++k) {
      const double* x0 = &s.xyz[3 * s.tet[4 * k]];
      const double* Ai = &s.Ainv[9 * k];
      double r[3];
      for (int i = 0; i < 3; ++i)
        r[i] = Ai[3 * i] * (dp.pos[0] - x0[0]) + Ai[3 * i + 1] * (dp.pos[1] - x0[1]) +
               Ai[3 * i + 2] * (dp.pos[2] - x0[2]);
      const double tol = -1e-12;
      if (r[0] >= tol && r[1] >= tol && r[2] >= tol && 1 - r[0] - r[1] - r[2] >= tol) {
        dp.elem = k;
        std::memcpy(rh, r, sizeof rh);
      }
    }
    if (dp.elem < 0) throw Error(MDG_E_ARG, "set_dipoles: point outside the mesh (or its instance)");
    dubiner3<double>(s.P, rh[0], rh[1], rh[2], val.data(), nullptr);
    const double* Ai = &s.Ainv[9 * dp.elem];
    double ad[3];
    for (int i = 0; i < 3; ++i) ad[i] = Ai[3 * i] * dp.dir[0] + Ai[3 * i + 1] * dp.dir[1] + Ai[3 * i + 2] * dp.dir[2];
    dp.coef.resize(3 * s.N);
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l < s.N; ++l) dp.coef[j * s.N + l] = val[l] * ad[j];
    out.push_back(dp);
  }
  s.dips = out;
  s.finalized = false;
  s.bound = false;
}

LdsLayout stage_lds_layout(const Solver& s, bool compact) {
  // reals: in-tile trace slots [0, T) (the publication stages the output in
  // [0, ST)), the staged input [SB, SB + ST), the halo slots from HB; plus 16
  // bytes of slack for the 16-byte granules of the halo copy
  const int rs = (int)s.real_size();
  const size_t ss = compact ? 2ull * s.NF + 1 : 4ull * s.NF + 1;
  const size_t T = 4ull * s.tile * ss;
  const size_t ST = (compact ? 1ull : 2ull) * 3ull * s.N * s.tile;
  const size_t H = (compact ? 1ull : 2ull) * (size_t)halo_role_reals(s.NF, rs) * (size_t)s.hmax;
  LdsLayout shared{0, (int32_t)std::max(T, ST), 0, 0}, beside{(int32_t)ST, (int32_t)std::max(T, 2 * ST), 0, 0};
  shared.bytes = (size_t(shared.halo_base) + H) * rs + 16;
  beside.bytes = (size_t(beside.halo_base) + H) * rs + 16;
  // the publication stages the output beside the trace slots (the input and
  // halo areas are dead by then) when that fits the same allocation
  for (LdsLayout* l : {&shared, &beside})
    if ((T + ST) * rs + 16 <= l->bytes) l->out_base = (int32_t)T;
  // workgroups per CU: by LDS, and by the register budget the kernel is
  // compiled for (waves per SIMD: FP32 4, or 3 at order 4; FP64 2)
  const int wpe = s.opt.precision == MDG_FP32 ? (s.P >= 4 ? 3 : 4) : 2;
  const int wg_waves = std::max(1, (compact ? 4 : 8) * s.tile / 64);
  const size_t by_regs = (size_t)std::max(1, 4 * wpe / wg_waves);
  auto per_cu = [&](size_t b) { return std::min(LDS_MAX_BYTES / b, by_regs); };
  // the input beside the output staging lets a workgroup copy its next
  // tile's input while publishing; take it unless it costs occupancy
  return per_cu(beside.bytes) >= per_cu(shared.bytes) ? beside : shared;
}

size_t stage_lds_bytes(const Solver& s) { return stage_lds_layout(s, false).bytes; }

size_t lf_lds_bytes(const Solver& s) { return stage_lds_layout(s, true).bytes; }

int tile_size_for(int P, bool fp32) {
  // elements per workgroup (eight lanes each: 2 fields x 4 parts, so 2*tile
  // must be a multiple of the 64-lane wave); the trace exchange in LDS needs
  // (4 NF + 1) (4 tile + halo) reals, kept under 64 KiB
  const int NF = nmodes2(P);
  const int rs = fp32 ? 4 : 8;
  for (int t : {64, 32}) {
    const double est = (4.0 * NF + 1) * (4.0 * t + 1.6 * t) * rs;
    if (est <= 60000.0) return t;
  }
  return 32;
}

// Tile order: recursive coordinate bisection of the element centroids over
// perm[b, e). A range is cut at the median of its longest centroid extent,
// with the cut moved to the tile boundary (o + a multiple of `leaf`, o the
// start of the tiled partition) nearest to the middle, until it holds no such multiple; that last range is
// sorted along its longest extent, so that halving the tile later still
// gives compact halves. Consecutive runs of `leaf` elements are then compact
// boxes, with fewer faces on their boundary (fewer halo traces) than runs of
// a space-filling curve, which follow octree cells only at powers of two.
static void bisect(std::vector<int64_t>& perm, int64_t b, int64_t e, int64_t o, int64_t leaf,
                   const std::vector<double>& cen) {
  while (e - b > 1) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = b; i < e; ++i)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], cen[3 * perm[i] + c]);
        hi[c] = std::max(hi[c], cen[3 * perm[i] + c]);
      }
    int ax = 0;
    for (int c = 1; c < 3; ++c)
      if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
    auto less = [&](int64_t x, int64_t y) { return cen[3 * x + ax] < cen[3 * y + ax]; };
    // tile boundaries inside (b, e)
    const int64_t first = o + (b - o) / leaf * leaf + leaf, last = o + (e - 1 - o) / leaf * leaf;
    if (first > last) {
      std::sort(perm.begin() + b, perm.begin() + e, less);
      return;
    }
    const int64_t m = std::min(last, std::max(first, o + ((b + e) / 2 - o + leaf / 2) / leaf * leaf));
    std::nth_element(perm.begin() + b, perm.begin() + m, perm.begin() + e, less);
    bisect(perm, b, m, o, leaf, cen);
    b = m;
  }
}

static uint64_t spread21(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// Halo slots of the tiles of perm[b, e) (runs of `leaf` from o): the largest
// count of faces of one tile whose neighbour lies in another tile, and the
// total. tile_of is scratch (all -1 on entry and on return).
static std::pair<int64_t, int64_t> halo_counts(const Solver& s, const std::vector<int64_t>& perm, int64_t b, int64_t e,
                                               int64_t o, int64_t leaf, std::vector<int64_t>& tile_of) {
  for (int64_t i = b; i < e; ++i) tile_of[perm[i]] = (i - o) / leaf;
  std::vector<int64_t> cnt((e - 1 - o) / leaf - (b - o) / leaf + 1, 0);
  int64_t total = 0;
  for (int64_t i = b; i < e; ++i) {
    const int64_t ku = perm[i], t = tile_of[ku];
    for (int f = 0; f < 4; ++f) {
      const int64_t sd = s.side[4 * ku + f];
      if (sd >= 0 && tile_of[sd / 4] != t) {
        ++cnt[t - (b - o) / leaf];
        ++total;
      }
    }
  }
  for (int64_t i = b; i < e; ++i) tile_of[perm[i]] = -1;
  return {*std::max_element(cnt.begin(), cnt.end()), total};
}

// Refines the tiles of perm[b, e) (runs of `leaf` from o) by swapping
// elements between face-adjacent tiles. Every element offers a move to each
// tile it touches, with the gain (its faces into that tile minus its faces
// into its own); the offers between two tiles are paired best first in both
// directions, and a pair is swapped when the gains recomputed at that moment
// (less 2 if the two are neighbours) add up to a positive number, so every
// swap removes cross-tile faces and tile sizes stay fixed. Sweeps repeat
// while they gain; the result is kept only if its largest halo block is not
// larger than the starting one. Each tile's elements are then sorted along
// its longest centroid extent (halving a tile still gives compact halves).
static void refine_tiles(const Solver& s, std::vector<int64_t>& perm, int64_t b, int64_t e, int64_t o, int64_t leaf,
                         const std::vector<double>& cen, std::vector<int64_t>& tile_of) {
  if (e - b <= leaf) return;
  const std::vector<int64_t> start(perm.begin() + b, perm.begin() + e);
  const int64_t max0 = halo_counts(s, perm, b, e, o, leaf, tile_of).first;
  struct Move {
    int64_t a, t, gain, i;  // from tile a to tile t, the element at position i
  };
  // faces of element x into tile t (t = its own tile: the faces kept inside)
  auto faces_into = [&](int64_t x, int64_t t) {
    int64_t c = 0;
    for (int f = 0; f < 4; ++f) {
      const int64_t sd = s.side[4 * x + f];
      c += sd >= 0 && tile_of[sd / 4] == t;
    }
    return c;
  };
  auto order = [](const Move& p, const Move& q) {
    if (p.a != q.a) return p.a < q.a;
    if (p.t != q.t) return p.t < q.t;
    return p.gain > q.gain;
  };
  std::vector<Move> moves;
  for (int sweep = 0; sweep < 16; ++sweep) {
    for (int64_t i = b; i < e; ++i) tile_of[perm[i]] = (i - o) / leaf;
    moves.clear();
    for (int64_t i = b; i < e; ++i) {
      const int64_t x = perm[i], a = tile_of[x], own = faces_into(x, a);
      for (int f = 0; f < 4; ++f) {
        const int64_t sd = s.side[4 * x + f];
        if (sd < 0) continue;
        const int64_t t = tile_of[sd / 4];
        if (t < 0 || t == a) continue;  // another group, or inside
        bool seen = false;
        for (int g = 0; g < f; ++g) seen = seen || (s.side[4 * x + g] >= 0 && tile_of[s.side[4 * x + g] / 4] == t);
        if (!seen) moves.push_back({a, t, faces_into(x, t) - own, i});
      }
    }
    std::sort(moves.begin(), moves.end(), order);
    int64_t swaps = 0;
    for (size_t k = 0; k < moves.size();) {
      const int64_t a = moves[k].a, t = moves[k].t;
      size_t k1 = k;
      while (k1 < moves.size() && moves[k1].a == a && moves[k1].t == t) ++k1;
      if (a < t) {
        auto q = std::lower_bound(moves.begin(), moves.end(), Move{t, a, INT64_MAX, 0}, order);
        for (size_t p = k; p < k1 && q != moves.end() && q->a == t && q->t == a;) {
          const int64_t xa = perm[moves[p].i], xb = perm[q->i];
          if (tile_of[xa] != a) { ++p; continue; }  // moved already
          if (tile_of[xb] != t) { ++q; continue; }
          bool adj = false;
          for (int f = 0; f < 4; ++f) adj = adj || (s.side[4 * xa + f] >= 0 && s.side[4 * xa + f] / 4 == xb);
          const int64_t g = faces_into(xa, t) - faces_into(xa, a) + faces_into(xb, a) - faces_into(xb, t) -
                            (adj ? 2 : 0);
          if (g <= 0) {
            if (moves[p].gain + q->gain <= 0) break;  // the remaining offers gain less
            if (moves[p].gain >= q->gain) ++q; else ++p;
            continue;
          }
          std::swap(perm[moves[p].i], perm[q->i]);
          tile_of[xa] = t;
          tile_of[xb] = a;
          ++swaps;
          ++p;
          ++q;
        }
      }
      k = k1;
    }
    for (int64_t i = b; i < e; ++i) tile_of[perm[i]] = -1;
    if (swaps == 0) break;
  }
  if (halo_counts(s, perm, b, e, o, leaf, tile_of).first > max0) {
    std::copy(start.begin(), start.end(), perm.begin() + b);
    return;
  }
  // compact halves inside every tile
  for (int64_t t0 = b; t0 < e;) {
    const int64_t t1 = std::min(e, o + ((t0 - o) / leaf + 1) * leaf);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = t0; i < t1; ++i)
      for (int c = 0; c < 3; ++c) {
        lo[c] = std::min(lo[c], cen[3 * perm[i] + c]);
        hi[c] = std::max(hi[c], cen[3 * perm[i] + c]);
      }
    int ax = 0;
    for (int c = 1; c < 3; ++c)
      if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
    std::sort(perm.begin() + t0, perm.begin() + t1,
              [&](int64_t x, int64_t y) { return cen[3 * x + ax] < cen[3 * y + ax]; });
    t0 = t1;
  }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void finalize(Solver& s) {
  if (s.nt == 0) throw Error(MDG_E_STATE, "no mesh");
  const int64_t nt = s.nt;
  std::vector<char> ispml(nt, 0);
  if (!s.omega.empty())
    for (int64_t k = 0; k < nt; ++k)
      ispml[k] = (s.omega[3 * k] > 0 || s.omega[3 * k + 1] > 0 || s.omega[3 * k + 2] > 0);
  const bool fp32 = s.opt.precision == MDG_FP32;
  const size_t rs = s.real_size();
  int tile0 = tile_size_for(s.P, fp32);
  // leap-frog: 64-element tiles let the half steps give all lanes to the
  // active field (the operator calls then may use a larger workgroup LDS)
  const bool lf = s.opt.integrator == MDG_LEAPFROG;
  if (lf) tile0 = 64;
  const bool forced = s.opt.tile != 0;  // a caller's choice (e.g. an autotuner)
  if (forced) tile0 = s.opt.tile;
  // non-PML elements, then PML elements; inside each, instance by instance,
  // each in the bisection order of its centroids (leaves of the first tile
  // size tried) or along its Morton curve, whichever gives the smaller
  // largest halo block (it sizes every workgroup's LDS), then the fewer halo
  // slots: bisection cuts compact boxes out of a convex region, but leaves
  // of a hollow one (a PML shell) can hold elements from both sides of the
  // hole; then refined by swaps between adjacent tiles
  std::vector<double> cen(3 * nt);
  for (int64_t k = 0; k < nt; ++k)
    for (int c = 0; c < 3; ++c) {
      double m = 0;
      for (int v = 0; v < 4; ++v) m += s.xyz[3 * s.tet[4 * k + v] + c];
      cen[3 * k + c] = 0.25 * m;
    }
  s.perm.resize(nt);
  std::iota(s.perm.begin(), s.perm.end(), 0);
  std::stable_sort(s.perm.begin(), s.perm.end(), [&](int64_t a, int64_t b) {
    if (ispml[a] != ispml[b]) return ispml[a] < ispml[b];
    return s.inst_of[a] < s.inst_of[b];
  });
  s.K = nt;
  s.K0 = 0;
  for (int64_t k = 0; k < nt; ++k) s.K0 += !ispml[k];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t k = 0; k < nt; ++k)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], cen[3 * k + c]);
      hi[c] = std::max(hi[c], cen[3 * k + c]);
    }
  std::vector<uint64_t> mkey(nt);
  for (int64_t k = 0; k < nt; ++k) {
    uint64_t code = 0;
    for (int c = 0; c < 3; ++c) {
      const double span = std::max(hi[c] - lo[c], 1e-300);
      code |= spread21((uint64_t)std::min(2097151.0, std::max(0.0, (cen[3 * k + c] - lo[c]) / span * 2097151.0))) << c;
    }
    mkey[k] = code;
  }
  std::vector<int64_t> tile_of(nt, -1), morton(nt);
  for (int64_t g0 = 0; g0 < nt;) {
    int64_t g1 = g0 + 1;
    while (g1 < nt && ispml[s.perm[g1]] == ispml[s.perm[g0]] && s.inst_of[s.perm[g1]] == s.inst_of[s.perm[g0]]) ++g1;
    const int64_t o = ispml[s.perm[g0]] ? s.K0 : 0;  // the damped partition is tiled from K0 on
    std::copy(s.perm.begin() + g0, s.perm.begin() + g1, morton.begin() + g0);
    std::stable_sort(morton.begin() + g0, morton.begin() + g1, [&](int64_t x, int64_t y) { return mkey[x] < mkey[y]; });
    bisect(s.perm, g0, g1, o, tile0, cen);
    if (halo_counts(s, morton, g0, g1, o, tile0, tile_of) < halo_counts(s, s.perm, g0, g1, o, tile0, tile_of))
      std::copy(morton.begin() + g0, morton.begin() + g1, s.perm.begin() + g0);
    refine_tiles(s, s.perm, g0, g1, o, tile0, cen, tile_of);
    g0 = g1;
  }
  s.iperm.resize(nt);
  for (int64_t k = 0; k < nt; ++k) s.iperm[s.perm[k]] = k;
  s.Kp = nt - s.K0;
  s.Kppad = (std::max<int64_t>(s.Kp, 1) + 63) / 64 * 64;

  for (int tile = tile0;; tile /= 2) {
    s.tile = tile;
    // padded by a full tile: lanes past the end of a partial tile load freely
    s.Kpad = (nt + tile + 63) / 64 * 64;
    s.tile_start.clear();
    s.tile_count.clear();
    for (int part = 0; part < 2; ++part) {
      const int64_t b = part == 0 ? 0 : s.K0, e = part == 0 ? s.K0 : s.K;
      for (int64_t x = b; x < e; x += tile) {
        s.tile_start.push_back((int32_t)x);
        s.tile_count.push_back((int32_t)std::min<int64_t>(tile, e - x));
      }
      if (part == 0) s.ntiles0 = (int64_t)s.tile_start.size();
    }
    s.ntiles = (int64_t)s.tile_start.size();
    // Connectivity codes and halo traces. A face whose neighbour lies in the
    // same tile is coded by the neighbour's trace slot (face * tile + index);
    // a face whose neighbour lies in another tile by a halo slot 4 tile + h.
    // The traces for halo slot h of tile t are written, one stage earlier, by
    // the neighbour itself into tile t's block of the halo buffer, at the
    // offset recorded in the neighbour's publish code.
    s.nbr_code.assign(4 * s.Kpad, -1);
    s.nbr_glob.assign(4 * s.Kpad, -1);
    for (int64_t k = 0; k < s.K; ++k)
      for (int f = 0; f < 4; ++f) {
        const int64_t sd = s.side[4 * s.perm[k] + f];
        if (sd >= 0) s.nbr_glob[4 * k + f] = (int32_t)(4 * s.iperm[sd / 4] + sd % 4);
      }
    s.pub_code.assign(4 * s.Kpad, -1);
    auto NB = [&](int f, int64_t k) -> int32_t& { return s.nbr_code[blk_index(k, f, 4)]; };
    auto PUB = [&](int f, int64_t k) -> int32_t& { return s.pub_code[blk_index(k, f, 4)]; };
    s.halo_tile.assign(2 * s.ntiles, 0);
    s.hmax = 0;
    s.nhalo = 0;
    // one region per reading role, each a sequence of per-tile blocks of
    // SH reals per slot; a pub code is the slot's offset inside a region
    const int64_t SH = halo_role_reals(s.NF, (int)rs);
    const int64_t align = 64 / (int64_t)rs;  // halo blocks start on 64-byte boundaries
    int64_t hoff = 0;
    struct HE { int32_t fn; int64_t kn; int64_t k; int f; };
    std::vector<HE> ents;
    for (int64_t t = 0; t < s.ntiles; ++t) {
      const int64_t b = s.tile_start[t], c = s.tile_count[t];
      ents.clear();
      for (int64_t k = b; k < b + c; ++k) {
        const int64_t ku = s.perm[k];
        for (int f = 0; f < 4; ++f) {
          const int64_t sd = s.side[4 * ku + f];
          if (sd < 0) continue;  // PEC
          const int64_t kn = s.iperm[sd / 4];
          const int fn = (int)(sd % 4);
          if (kn >= b && kn < b + c)
            NB(f, k) = (int32_t)(fn * tile + (kn - b));
          else
            ents.push_back({fn, kn, k, f});
        }
      }
      std::stable_sort(ents.begin(), ents.end(), [](const HE& x, const HE& y) {
        if (x.kn != y.kn) return x.kn < y.kn;
        return x.fn < y.fn;
      });
      for (size_t h = 0; h < ents.size(); ++h) {
        NB(ents[h].f, ents[h].k) = (int32_t)(4 * tile + h);
        PUB(ents[h].fn, ents[h].kn) = (int32_t)(hoff + (int64_t)h * SH);
      }
      const int64_t nh = (int64_t)ents.size();
      s.halo_tile[2 * t] = (int32_t)hoff;
      s.halo_tile[2 * t + 1] = (int32_t)nh;
      hoff = (hoff + nh * SH + align - 1) / align * align;
      if (hoff >= (int64_t(1) << 31)) throw Error(MDG_E_UNSUPPORTED, "mesh too large: halo buffer exceeds 2^31 reals");
      s.nhalo += nh;
      s.hmax = std::max<int>(s.hmax, (int)nh);
    }
    s.hreg = std::max<int64_t>(hoff, align);
    s.hbuf_reals = 2 * s.hreg;
    const size_t lds = stage_lds_bytes(s);
    // the default choice keeps two workgroups per CU; a forced tile only has
    // to fit the LDS of one workgroup
    if (lds <= LDS_MAX_BYTES / 2 || (forced && lds <= LDS_MAX_BYTES)) break;
    if (lf && tile == 64 && lf_lds_bytes(s) <= LDS_MAX_BYTES / 2 && lds <= LDS_MAX_BYTES) break;
    if (tile <= 32) {
      // up to 160 KiB per workgroup on gfx950 (checked against the device at bind time)
      if (lds <= LDS_MAX_BYTES) break;
      throw Error(MDG_E_UNSUPPORTED, "face-trace exchange does not fit in the LDS of one workgroup");
    }
  }
  if (s.K >= (int64_t(1) << 29)) throw Error(MDG_E_ARG, "mesh too large");
  if (size_t(s.hbuf_reals) * rs >= (size_t(1) << 32)) throw Error(MDG_E_UNSUPPORTED, "mesh too large: halo buffer exceeds 4 GiB");

  // geometry records
  s.geo.assign(size_t(NGEO) * s.Kpad, 0.0);
  auto G = [&](int row, int64_t k) -> double& { return s.geo[blk_index(k, row, NGEO)]; };
  for (int64_t k = 0; k < s.Kpad; ++k) {
    if (k >= s.K) {  // padding: harmless values
      G(G_XX, k) = G(G_YY, k) = G(G_ZZ, k) = 1.0;
      G(G_IEPS, k) = G(G_IMU, k) = G(G_SIGN, k) = G(G_Z, k) = 1.0;
      for (int f = 0; f < 4; ++f) G(G_WZ0 + f, k) = 0.5;
      continue;
    }
    const int64_t u = s.perm[k];
    const double* A = &s.A[9 * u];
    const double J = std::fabs(s.det[u]);
    double AtA[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int r = 0; r < 3; ++r) v += A[3 * r + i] * A[3 * r + j];
        AtA[3 * i + j] = v / J;
      }
    G(G_XX, k) = AtA[0];
    G(G_XY, k) = AtA[1];
    G(G_XZ, k) = AtA[2];
    G(G_YY, k) = AtA[4];
    G(G_YZ, k) = AtA[5];
    G(G_ZZ, k) = AtA[8];
    G(G_IEPS, k) = 1.0 / s.eps[u];
    G(G_IMU, k) = 1.0 / s.mu[u];
    G(G_SIGN, k) = s.det[u] > 0 ? 1.0 : -1.0;
    const double Zm = std::sqrt(s.mu[u] / s.eps[u]);
    G(G_Z, k) = Zm;
    for (int f = 0; f < 4; ++f) {
      const int64_t sd = s.side[4 * u + f];
      if (sd < 0) {
        G(G_WZ0 + f, k) = 0.5;
      } else {
        const int64_t un = sd / 4;
        const double Zp = std::sqrt(s.mu[un] / s.eps[un]);
        G(G_WZ0 + f, k) = Zm / (Zm + Zp);
      }
    }
    if (s.sip()) {
      // alpha_F / mu_F of each face: alpha_F = alpha0 (p+1)(p+3)/3 |F| / min(|T|, |T'|),
      // mu_F the mean of the two sides (the element's own on PEC faces); both
      // sides evaluate the same expression in the same order
      const int p = s.P;
      for (int f = 0; f < 4; ++f) {
        const int64_t sd = s.side[4 * u + f];
        int fv[3];
        face_vertices(f, fv);
        const double* xa = &s.xyz[3 * s.tet[4 * u + fv[0]]];
        const double* xb = &s.xyz[3 * s.tet[4 * u + fv[1]]];
        const double* xc = &s.xyz[3 * s.tet[4 * u + fv[2]]];
        double t1[3], t2[3];
        for (int i = 0; i < 3; ++i) { t1[i] = xb[i] - xa[i]; t2[i] = xc[i] - xa[i]; }
        const double cx = t1[1] * t2[2] - t1[2] * t2[1], cy = t1[2] * t2[0] - t1[0] * t2[2],
                     cz = t1[0] * t2[1] - t1[1] * t2[0];
        const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        const double vm = std::fabs(s.det[u]) / 6.0;
        const double vo = sd < 0 ? vm : std::fabs(s.det[sd / 4]) / 6.0;
        const double alpha = s.opt.sip_alpha * (p + 1) * (p + 3) / 3.0 * area / std::min(vm, vo);
        const double muF = sd < 0 ? s.mu[u] : 0.5 * (s.mu[u] + s.mu[sd / 4]);
        G(G_SIP0 + f, k) = alpha / muF;
      }
    }
  }
  // PML records: A^T, A^-T (row-major) and the damping
  s.pmlrec.assign(size_t(NPML) * s.Kppad, 0.0);
  for (int64_t k = s.K0; k < s.K; ++k) {
    const int64_t u = s.perm[k], pk = k - s.K0;
    const double* A = &s.A[9 * u];
    const double* Ai = &s.Ainv[9 * u];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        s.pmlrec[blk_index(pk, PM_AT + 3 * i + j, NPML)] = A[3 * j + i];
        s.pmlrec[blk_index(pk, PM_AIT + 3 * i + j, NPML)] = Ai[3 * j + i];
      }
    for (int c = 0; c < 3; ++c) s.pmlrec[blk_index(pk, PM_OM + c, NPML)] = s.omega[3 * u + c];
  }
  // device layout
  DevLayout& L = s.L;
  size_t off = 0;
  const size_t field = size_t(state_rows(s)) * s.Kpad * rs;
  const size_t afield = s.Kp > 0 ? size_t(state_rows(s)) * s.Kppad * rs : 0;
  L.Y = off; off = align256(off + field);
  L.Ua = off; off = align256(off + field);
  L.Ub = off; off = align256(off + field);
  L.ACC = off; off = align256(off + field);
  L.aY = off; off = align256(off + afield);
  L.aUa = off; off = align256(off + afield);
  L.aUb = off; off = align256(off + afield);
  L.aACC = off; off = align256(off + afield);
  const size_t sfield = s.sip() ? size_t(8) * s.NF * s.Kpad * rs : 0;
  L.sY = off; off = align256(off + sfield);
  L.sUa = off; off = align256(off + sfield);
  L.sUb = off; off = align256(off + sfield);
  L.sACC = off; off = align256(off + sfield);
  L.geo = off; off = align256(off + size_t(NGEO) * s.Kpad * rs);
  L.nbr = off; off = align256(off + size_t(4) * s.Kpad * 4);
  L.nbrg = off; off = align256(off + size_t(4) * s.Kpad * 4);
  L.pub = off; off = align256(off + size_t(4) * s.Kpad * 4);
  L.halo_tile = off; off = align256(off + size_t(2) * s.ntiles * 4);
  L.H0 = off; off = align256(off + size_t(s.hbuf_reals) * rs);
  L.H1 = off; off = align256(off + size_t(s.hbuf_reals) * rs);
  L.pml = off; off = align256(off + (s.Kp > 0 ? size_t(NPML) * s.Kppad * rs : 0));
  const size_t ndip = std::max<size_t>(s.dips.size(), 1);
  L.src = off; off = align256(off + ndip * 3 * s.N * rs);
  L.srcid = off; off = align256(off + size_t(s.Kpad) * 4);
  L.srcnext = off; off = align256(off + ndip * 4);
  L.srcwave = off; off = align256(off + ndip * 3 * 8);
  L.srcamp = off; off = align256(off + 4 * ndip * 8);  // [RK4 stage][dipole]
  L.clock = off; off = align256(off + 2 * 8);
  L.rhs_clock = off; off = align256(off + 2 * 8);
  L.eelem = off; off = align256(off + size_t(s.K) * 8);
  const size_t nblk = (s.K + 255) / 256;
  L.epart = off; off = align256(off + nblk * 8);
  L.eout = off; off = align256(off + 8);
  L.mon = off; off = align256(off + 4 * 8);
  L.total = off;
  s.finalized = true;
}

double cfl_dt(const Solver& s) {
  // dt = cfl * min_T (2 r_in sqrt(eps mu)) / (p+1)^2, r_in = 3|T| / sum |faces|
  double best = 1e300;
  for (int64_t k = 0; k < s.nt; ++k) {
    const int64_t* t = &s.tet[4 * k];
    double area = 0;
    for (int f = 0; f < 4; ++f) {
      int fv[3];
      face_vertices(f, fv);
      const double* a = &s.xyz[3 * t[fv[0]]];
      const double* b = &s.xyz[3 * t[fv[1]]];
      const double* c = &s.xyz[3 * t[fv[2]]];
      double u[3], v[3];
      for (int i = 0; i < 3; ++i) { u[i] = b[i] - a[i]; v[i] = c[i] - a[i]; }
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
                   cz = u[0] * v[1] - u[1] * v[0];
      area += 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    }
    const double vol = std::fabs(s.det[k]) / 6.0;
    const double rin = 3.0 * vol / area;
    best = std::min(best, 2.0 * rin * std::sqrt(s.eps[k] * s.mu[k]));
  }
  return s.opt.cfl * best / double((s.P + 1) * (s.P + 1));
}

void projection_points(const Solver& s, int q, double* xyz) {
  std::vector<double> pts, w;
  tet_rule<double>(q, pts, w);
  const size_t Q = w.size();
  for (int64_t k = 0; k < s.nt; ++k) {
    const double* x0 = &s.xyz[3 * s.tet[4 * k]];
    const double* A = &s.A[9 * k];
    for (size_t i = 0; i < Q; ++i)
      for (int r = 0; r < 3; ++r)
        xyz[(k * Q + i) * 3 + r] =
            x0[r] + A[3 * r] * pts[3 * i] + A[3 * r + 1] * pts[3 * i + 1] + A[3 * r + 2] * pts[3 * i + 2];
  }
}

void project_fields(const Solver& s, int q, const double* vals, int N, std::vector<double>& coef) {
  // Cartesian L2 projection c_l = (1/|det A|) int_T F phi_l = sum_q w_q F(x_q) phi^_l(r^_q),
  // then covariant coefficients u_l = A^T c_l, for the first N modes (the
  // projection onto a lower order space is the truncation: orthonormal,
  // degree-ordered modes)
  std::vector<double> pts, w;
  tet_rule<double>(q, pts, w);
  const size_t Q = w.size();
  const int NP = s.N;
  std::vector<double> phall(NP), phi(Q * N);
  for (size_t i = 0; i < Q; ++i) {
    dubiner3<double>(s.P, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], phall.data(), nullptr);
    for (int l = 0; l < N; ++l) phi[i * N + l] = phall[l];
  }
  coef.assign(size_t(s.nt) * 3 * N, 0.0);
  std::vector<double> c(3 * N);
  for (int64_t k = 0; k < s.nt; ++k) {
    std::fill(c.begin(), c.end(), 0.0);
    for (size_t i = 0; i < Q; ++i) {
      const double* F = &vals[(k * Q + i) * 3];
      for (int r = 0; r < 3; ++r)
        for (int l = 0; l < N; ++l) c[r * N + l] += w[i] * F[r] * phi[i * N + l];
    }
    const double* A = &s.A[9 * k];
    for (int j = 0; j < 3; ++j)
      for (int l = 0; l < N; ++l)
        coef[(k * 3 + j) * N + l] = A[j] * c[l] + A[3 + j] * c[N + l] + A[6 + j] * c[2 * N + l];
  }
}

// host arrays: E [nt][3][N], H [nt][3][NH]; device rows state_row
void pack_state(const Solver& s, const double* E, const double* H, std::vector<double>& out) {
  const int N = s.N, NH = s.NH, RB = state_rows(s);
  out.assign(size_t(RB) * s.Kpad, 0.0);
  for (int64_t k = 0; k < s.K; ++k) {
    const int64_t u = s.perm[k];
    for (int c = 0; c < 3; ++c) {
      if (E)
        for (int l = 0; l < N; ++l) out[blk_index(k, state_row(s, 0, c, l), RB)] = E[(u * 3 + c) * N + l];
      if (H)
        for (int l = 0; l < NH; ++l) out[blk_index(k, state_row(s, 1, c, l), RB)] = H[(u * 3 + c) * NH + l];
    }
  }
}

void unpack_state(const Solver& s, const std::vector<double>& in, double* E, double* H) {
  const int N = s.N, NH = s.NH, RB = state_rows(s);
  for (int64_t k = 0; k < s.K; ++k) {
    const int64_t u = s.perm[k];
    for (int c = 0; c < 3; ++c) {
      if (E)
        for (int l = 0; l < N; ++l) E[(u * 3 + c) * N + l] = in[blk_index(k, state_row(s, 0, c, l), RB)];
      if (H)
        for (int l = 0; l < NH; ++l) H[(u * 3 + c) * NH + l] = in[blk_index(k, state_row(s, 1, c, l), RB)];
    }
  }
}

void pack_aux(const Solver& s, const double* P, const double* Q, std::vector<double>& out) {
  // internal auxiliary = A^-T P / eps (Cartesian, scaled): the PML terms then
  // need no material factor inside the kernel
  const int N = s.N, RB = state_rows(s);
  out.assign(size_t(RB) * s.Kppad, 0.0);
  for (int which = 0; which < 2; ++which) {
    const double* in = which == 0 ? P : Q;
    if (!in) continue;
    const int Nw = which == 0 ? N : s.NH;  // host modes of this field
    for (int64_t k = s.K0; k < s.K; ++k) {
      const int64_t u = s.perm[k], pk = k - s.K0;
      const double* Ai = &s.Ainv[9 * u];
      const double m = which == 0 ? s.eps[u] : s.mu[u];
      for (int l = 0; l < Nw; ++l)
        for (int j = 0; j < 3; ++j) {
          double v = 0;
          for (int i = 0; i < 3; ++i) v += Ai[3 * i + j] * in[(u * 3 + i) * Nw + l];
          out[blk_index(pk, state_row(s, which, j, l), RB)] = v / m;
        }
    }
  }
}

void unpack_aux(const Solver& s, const std::vector<double>& in, double* P, double* Q) {
  const int N = s.N, RB = state_rows(s);
  for (int which = 0; which < 2; ++which) {
    double* out = which == 0 ? P : Q;
    if (!out) continue;
    const int Nw = which == 0 ? N : s.NH;
    std::fill(out, out + size_t(s.nt) * 3 * Nw, 0.0);
    for (int64_t k = s.K0; k < s.K; ++k) {
      const int64_t u = s.perm[k], pk = k - s.K0;
      const double* A = &s.A[9 * u];
      const double m = which == 0 ? s.eps[u] : s.mu[u];
      for (int l = 0; l < Nw; ++l)
        for (int j = 0; j < 3; ++j) {
          double v = 0;
          for (int i = 0; i < 3; ++i) v += A[3 * i + j] * in[blk_index(pk, state_row(s, which, i, l), RB)];
          out[(u * 3 + j) * Nw + l] = v * m;
        }
    }
  }
}

// host rows (face, k, m < NFH) <-> device rows (face * 2 + k) * NF + m; with
// mixed orders the face modes NFH.. of the kernel's order stay zero
void pack_sip(const Solver& s, const double* S, std::vector<double>& out) {
  const int R8 = 8 * s.NF, NFH = s.NFH;
  out.assign(size_t(R8) * s.Kpad, 0.0);
  if (!S) return;
  for (int64_t k = 0; k < s.K; ++k) {
    const int64_t u = s.perm[k];
    for (int fk = 0; fk < 8; ++fk)
      for (int m = 0; m < NFH; ++m) out[blk_index(k, fk * s.NF + m, R8)] = S[(u * 8 + fk) * NFH + m];
  }
}

void unpack_sip(const Solver& s, const std::vector<double>& in, double* S) {
  const int R8 = 8 * s.NF, NFH = s.NFH;
  for (int64_t k = 0; k < s.K; ++k) {
    const int64_t u = s.perm[k];
    for (int fk = 0; fk < 8; ++fk)
      for (int m = 0; m < NFH; ++m) S[(u * 8 + fk) * NFH + m] = in[blk_index(k, fk * s.NF + m, R8)];
  }
}

static void nnz_of(int P, int& nd, int& nf) {
  switch (P) {
    case 1: nd = ref::Ops<1>::nnzD; nf = ref::Ops<1>::nnzT; break;
    case 2: nd = ref::Ops<2>::nnzD; nf = ref::Ops<2>::nnzT; break;
    case 3: nd = ref::Ops<3>::nnzD; nf = ref::Ops<3>::nnzT; break;
    default: nd = ref::Ops<4>::nnzD; nf = ref::Ops<4>::nnzT; break;
  }
}

double bytes_per_stage(const Solver& s) {
  // classic RK4 with fused stages moves 17 state arrays per step (stage 1:
  // 1 read + 2 writes, stages 2-3: 3 reads + 2 writes, stage 4: 3 reads +
  // 1 write) -> 17/4 per stage; plus the geometry record and 4 neighbour codes
  // A leap-frog half step reads both fields and writes one (on average
  // 4.5 (N + NH) reals per element); a PML element reads and writes one
  // auxiliary field. With mixed orders only the NH modes of h count.
  const double rs = (double)s.real_size();
  const bool lf = s.opt.integrator == MDG_LEAPFROG;
  const double nn = double(s.N + s.NH);
  const double state = (lf ? 4.5 : 17.0 / 4.0 * 3.0) * nn * rs;
  const double geo = (s.opt.flux == MDG_UPWIND ? 14.0 : 9.0) * rs + 16.0;
  const double pml = (lf ? 3.0 : 17.0 / 4.0 * 3.0) * nn * rs + NPML * rs;
  // SIP: 8 NF surface values per element streamed like the state (the E
  // half of a leap-frog step reads them, the H half reads and writes them)
  // plus the four face rows of the geometry record
  const double sip = s.sip() ? (lf ? 12.0 : 17.0 / 4.0 * 8.0) * s.NFH * rs + 4.0 * rs : 0.0;
  return s.K * (state + geo + sip) + s.Kp * pml;
}

double flops_per_stage(const Solver& s) {
  int nd, nf;
  nnz_of(s.P, nd, nf);
  const double N = s.N, NF = s.NF;
  // per lane (two per element): traces 2 nf FMA, volume 2 nd FMA, lift 2 nf
  // FMA, flux per face, 3x3 mass per mode, RK epilogue
  const double flux = 4.0 * NF * (s.opt.flux == MDG_UPWIND ? 14.0 : 6.0);
  const double lane = 2.0 * (2.0 * nf + 2.0 * nd + 2.0 * nf) + flux + 18.0 * N + 4.0 * 3.0 * N;
  const double pml = 2.0 * N * 60.0;
  return 2.0 * lane * s.K + pml * s.Kp;
}

}  // namespace mdg

// solver.hpp -- internal state of a libmdg handle (host side) and the
// interfaces between host setup (setup.cpp), kernels (stage_kernel.hip) and
// the C ABI (api.hip).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mdg.h"

namespace mdg {

struct Error : std::runtime_error {
  mdg_status code;
  Error(mdg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// Per-element geometry record, one SoA row each (internal element order).
enum GeoRow {
  G_XX = 0, G_XY, G_XZ, G_YY, G_YZ, G_ZZ,  // G0^-1 = A^T A / |det A|
  G_IEPS,                                  // 1/eps
  G_IMU,                                   // 1/mu
  G_SIGN,                                  // sign(det A)
  G_Z,                                     // sqrt(mu/eps)
  G_WZ0, G_WZ1, G_WZ2, G_WZ3,              // Z-/(Z- + Z+) per local face (1/2 on PEC faces)
  NGEO
};
// With the SIP surface unknown (central flux only) the four face rows of the
// upwind weights hold alpha_F / mu_F of each local face instead.
constexpr int G_SIP0 = G_WZ0;
// Per-PML-element record rows.
enum PmlRow { PM_AT = 0, PM_AIT = 9, PM_OM = 18, NPML = 21 };

struct Dipole {
  double pos[3], dir[3], wave[3];  // wave = (f0, bw, t0)
  int32_t inst;                    // instance searched for the element (-1: whole mesh)
  int64_t elem;                    // user order
  std::vector<double> coef;        // [3][N] covariant load vector phi_l(r0) (A^-1 d)_j
};

// Device array layout: blocks of BLK = 64 consecutive elements ("AoSoA"),
// inside a block row-major over the per-element quantities, element fastest:
//   state  [K/64][field E,H][3N rows][64]    (row = component*N + mode)
//   geo    [K/64][NGEO][64],  nbr [K/64][4][64]
//   aux    [Kp/64][field P,Q][3N][64],  pml [Kp/64][NPML][64]
// A wave reads one row of 64 elements as one contiguous 256/512-byte segment;
// the field and the row of an access are small constant offsets.
constexpr int BLK = 64;
// Rows of one element in a state or auxiliary block: e (and p) with N modes
// per component, then h (and q) with NH modes (fewer than N with mixed
// orders): row c N + l of e, 3N + c NH + l of h.
struct Solver;
int state_rows(const Solver& s);
int state_row(const Solver& s, int field, int c, int l);
inline size_t blk_index(int64_t e, int row, int rows_per_block) {
  return (size_t(e / BLK) * rows_per_block + row) * BLK + size_t(e % BLK);
}

// Device buffer offsets (bytes into the workspace).
struct DevLayout {
  size_t Y, Ua, Ub, ACC;      // E and H together: [K/64][2][3N][64]
  size_t aY, aUa, aUb, aACC;  // PML auxiliaries P~, Q~: [Kp/64][2][3N][64]
  size_t sY, sUa, sUb, sACC;  // SIP surface unknown, one copy per element face: [K/64][4][2][NF][64]
  size_t geo, nbr, pub, halo_tile, pml;
  size_t nbrg;  // [Kpad][4] int32: neighbour element * 4 + its face, -1 = PEC (adjoint of the upwind flux)
  size_t src, srcid, srcnext, srcwave, srcamp;  // dipoles: coefficients, first dipole per element, chain,
                                                 // waveforms, amplitudes at the current stage
  size_t clock, rhs_clock;              // device time: (t0, n) of the stepping clock and of mdg_rhs
  size_t eelem;                         // per-element energies (FP64)
  size_t H0, H1;  // halo trace buffers: stage inputs' traces on cross-tile faces (ping-pong)
  size_t epart, eout;
  size_t mon;  // energy monitor of mdg_step: last energy, flag, first/last energies (FP64)
  size_t total;
};

struct Solver {
  mdg_options opt{};
  int P = 0, N = 0, NF = 0;  // order, modes and face modes of the kernel (of e)
  int NH = 0;                // modes of h: N, or dim P_{P-1} with mixed orders
  int NFH = 0;               // face modes of the SIP unknown (degree of h): NF, or dim P_{P-1}(F)
  std::string err;
  // ---- mesh (caller's element order, canonical vertex order)
  int64_t nv = 0, nt = 0;
  std::vector<double> xyz;
  std::vector<int64_t> tet;            // [nt][4], ascending ids
  std::vector<double> A, Ainv, det;    // [nt][9], [nt][9], [nt]
  std::vector<int64_t> side;           // [nt][4]: neighbour elem*4+face, or -1
  int64_t n_int = 0, n_bnd = 0;
  std::vector<double> eps, mu, omega;  // omega [nt][3] (empty = no PML)
  std::vector<Dipole> dips;
  std::vector<int64_t> inst_first;     // instance element ranges (caller order), size ninst + 1
  std::vector<int32_t> inst_of;        // [nt] instance of each element (caller order)
  // ---- decomposition (valid when finalized)
  bool finalized = false;
  int tile = 0;
  int64_t K = 0, K0 = 0, Kp = 0, Kpad = 0, Kppad = 0;
  std::vector<int64_t> perm;   // internal -> user
  std::vector<int64_t> iperm;  // user -> internal
  int64_t ntiles = 0, ntiles0 = 0, nhalo = 0;
  int hmax = 0;
  std::vector<int32_t> tile_start, tile_count;
  std::vector<int32_t> nbr_code;   // blocked [Kpad/64][4][64]: trace slot of the face's neighbour, -1 = PEC
  std::vector<int32_t> nbr_glob;   // [Kpad][4]: neighbour element * 4 + face (sorted order), -1 = PEC
  std::vector<int32_t> pub_code;   // blocked [Kpad/64][4][64]: halo-buffer offset (reals) of the face's trace, or -1
  std::vector<int32_t> halo_tile;  // [ntiles][2]: halo block offset (reals), halo slot count
  int64_t hbuf_reals = 0;         // both regions of one halo buffer
  int64_t hreg = 0;               // reals of one region (the traces one role reads)
  bool halo_valid = false;         // H0 holds the traces of Y
  std::vector<double> geo;     // blocked [Kpad/64][NGEO][64]
  std::vector<double> pmlrec;  // blocked [Kppad/64][NPML][64]
  // ---- device
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = false;
  bool bound = false;
  DevLayout L{};
  double t0 = 0.0, dt = 0.0;  // time of the last set state; the clock counts steps from it
  int64_t nstep = 0;
  double time() const { return t0 + double(nstep) * dt; }
  void* graph_exec = nullptr;  // hipGraphExec_t of graph_steps steps (mdg_step_graph)
  void* graph = nullptr;       // hipGraph_t
  int graph_steps = 0;
  size_t real_size() const { return opt.precision == MDG_FP32 ? 4 : 8; }
  bool sip() const { return opt.sip_alpha > 0; }
};

inline int state_rows(const Solver& s) { return 3 * (s.N + s.NH); }
inline int state_row(const Solver& s, int field, int c, int l) { return field == 0 ? c * s.N + l : 3 * s.N + c * s.NH + l; }

// ---- setup.cpp
void setup_mesh(Solver& s, int64_t nv, const double* xyz, int64_t nt, const int64_t* tet);
void setup_material(Solver& s, const double* eps, const double* mu);
void setup_pml(Solver& s, const double* omega);
void setup_instances(Solver& s, int n, const int64_t* first);
void setup_dipoles(Solver& s, int n, const int32_t* inst, const double* pos, const double* dir,
                   const double* wave);
void finalize(Solver& s);  // ordering, tiles, halo, geometry records, layout
double cfl_dt(const Solver& s);
int tile_size_for(int P, bool fp32);
// Halo trace slots: the two tangential traces of one field (2 NF reals) are
// padded to a multiple of 16 bytes (hrr reals), so every slot starts 16-byte
// aligned (the publishing lane writes it with 16-byte stores). The halo
// buffer holds one region per reading role; a tile's block in each region
// has one slot per halo face. In-tile slots keep the odd stride 4 NF + 1.
inline int halo_role_reals(int NF, int rs) { return (2 * NF * rs + 15) / 16 * 16 / rs; }
// LDS of one stage-kernel workgroup: offsets (reals) of the staged input
// field(s) and of the halo slots, and the bytes. compact: leap-frog halves
// with four lanes per element (64-element tiles: the input field staged,
// compact in-tile slots, the halo block of the active role only)
struct LdsLayout {
  int32_t stg_base, halo_base;
  size_t bytes;
  int32_t out_base;  // output staging of the publication beside the trace slots, or 0
};
LdsLayout stage_lds_layout(const Solver& s, bool compact);
// dynamic LDS of one stage-kernel workgroup: the face-trace exchange
size_t stage_lds_bytes(const Solver& s);
// leap-frog halves with four lanes per element (64-element tiles): the input
// field staged, compact in-tile slots, the same halo slots
size_t lf_lds_bytes(const Solver& s);
constexpr size_t LDS_MAX_BYTES = 160 * 1024;  // gfx950 LDS per workgroup
void projection_points(const Solver& s, int q, double* xyz);
void project_fields(const Solver& s, int q, const double* vals, int N, std::vector<double>& coef);
// state conversion between the caller's FP64 [nt][3][N] arrays and the
// internal blocked layout (as double); auxiliaries are stored as A^-T P / eps
// (P) and A^-T Q / mu (Q).
void pack_state(const Solver& s, const double* E, const double* H, std::vector<double>& out);
void unpack_state(const Solver& s, const std::vector<double>& in, double* E, double* H);
void pack_aux(const Solver& s, const double* P, const double* Q, std::vector<double>& out);
// SIP unknown: caller's S[nt][4][2][NFH] <-> blocked [Kpad/64][8 NF][64] (rows of modes >= NFH zero)
void pack_sip(const Solver& s, const double* S, std::vector<double>& out);
void unpack_sip(const Solver& s, const std::vector<double>& in, double* S);
void unpack_aux(const Solver& s, const std::vector<double>& in, double* P, double* Q);
double bytes_per_stage(const Solver& s);
double flops_per_stage(const Solver& s);

// ---- stage_kernel.hip
struct StageParams {
  int stage;      // 0..3 RK4 stage, -1 = operator output only, 4/5 leap-frog E/H half step
  double bcoef;   // b_i
  double cdt;     // c_{i+1} dt (stages 0..2)
  double dt;
  double cstage;  // c_i: the stage's time is clock t0 + (n + c_i) dt
  const double* clock;
  bool sources = true;    // add the dipole currents
  double* tick = nullptr;  // device clock to advance by one step in this launch
  // state buffers (E and H together, blocked layout); the final stage writes
  // the new state to Yout, or in place into Y when Yout is null
  void* Y;
  const void* Uin;
  void* Uout;
  void* ACC;
  void* aY;
  const void* aUin;
  void* aUout;
  void* aACC;
  // SIP surface unknown (ignored without it): base, stage input/output, accumulator
  void* sY = nullptr;
  const void* sUin = nullptr;
  void* sUout = nullptr;
  void* sACC = nullptr;
  void* Yout = nullptr;
  void* aYout = nullptr;
  void* sYout = nullptr;
  // non-null: the stage derivative k is stored there as well
  void* Kout = nullptr;
  void* aKout = nullptr;
  void* sKout = nullptr;
  // halo traces (see Solver::pub_code): read for the input, written for the output
  const void* hin;
  void* hout;
  bool publish;  // write the output's halo traces (false for the operator-only call)
  bool adj = false;  // operator calls: the adjoint operator in the mass inner product
};
void launch_stage(const Solver& s, const StageParams& sp, void* stream);
// halo traces of state U (blocked layout) into the halo buffer H
// (list: only the nlist listed elements, a device array of element indices)
void launch_publish(const Solver& s, const void* U, void* H, void* stream, const int64_t* list = nullptr,
                    int nlist = 0);
void launch_energy(const Solver& s, const void* Y, void* stream);
// energy monitor: after launch_energy, compare the energy with the last one
// recorded in mon (init: only record it); sets mon[1] to 1 on growth beyond
// the relative tolerance tol (if growth checks apply), 2 on a non-finite value
void launch_monitor(const Solver& s, bool init, bool growth, double tol, void* stream);

// ---- adjoint_kernel.hip (state vectors in the blocked layout, E and H)
void launch_probe_energy(const Solver& s, const void* u, const int64_t* probes, int np, double dt, double* J,
                         void* stream);  // J += dt sum_probes (e, e)_M0
void launch_probe_add(const Solver& s, void* nu, const void* u, const int64_t* probes, int np, double dt,
                      void* stream);  // nu_E += 2 dt / eps u_E on probes
// one forward stage: g -= scale (a, K)_M0,E, and on PML elements
// g -= scale (a, A^T (eta A^-T x_E + xa_E))_M0,E for the stage input
// (x, xa) + c (dx, dxa) (dx, dxa null: the stage input is (x, xa))
void launch_grad_stage(const Solver& s, double* g, const void* a, const void* K, const void* x, const void* dx,
                       const void* xa, const void* dxa, double c, double scale, void* stream);
// upwind flux: g += scale (a, dA/deps x) for the stage input x + c dx (dx may
// be null), the impedance dependence of the face terms (stage_kernel.hip,
// where the face operators live)
void launch_grad_upw(const Solver& s, double* g, const void* a, const void* x, const void* dx, double c,
                     double scale, void* stream);

}  // namespace mdg

/*
 * mdg.h -- C ABI of libmdg: matrix-free discontinuous Galerkin time-domain
 * Maxwell solver on tetrahedral meshes for AMD Instinct MI355X (gfx950).
 *
 * Method: Kapidani & Schoeberl, "A matrix-free Discontinuous Galerkin method
 * for the time dependent Maxwell equations in unbounded domains"
 * (arXiv:2002.08733). Cited below as [KS] with section / equation labels.
 *
 * What the library computes (the "hot path", one RK stage per kernel launch):
 *   eps d_t e = curl h - j,  mu d_t h = -curl e            [KS Sec. I, eqs. ampere_cont, faraday_cont]
 * discretised with element-wise P_p vector fields expanded in the covariantly
 * mapped orthonormal Dubiner basis A_T^-T e_j phi_l         [KS Sec. II, eq. mapped_eh]
 * so that the mass matrix is 3x3 block diagonal and the volume curl is one
 * geometry-independent reference matrix                    [KS Sec. III, eq. matrix_free_curl]
 * with central [KS Sec. III, eqs. uwc/cwc] or upwind numerical fluxes, PEC
 * boundaries [KS Sec. IV], complex-stretching PML auxiliary fields
 * [KS Sec. IV, eqs. p_variable, q_variable] and classic RK4 time stepping.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Element frame: the vertices of each tetrahedron are sorted by ascending
 *    global vertex id; v0 is the origin of the affine map r = A r^ + v0 with
 *    A = [v1-v0, v2-v0, v3-v0] (columns) [KS Sec. II, eq. mapping_template].
 *  - Field coefficients are *covariant* reference coefficients u[t][j][l]
 *    (element t in the caller's order, component j = 0..2, mode l = 0..N-1),
 *    so that e(r) = A_t^-T sum_l u[t][:][l] phi_l(A_t^-1 (r - v0)).
 *    N = (p+1)(p+2)(p+3)/6. Mode order: total degree d ascending, then the
 *    Dubiner index i, then j (phi_ijk as in [KS Sec. II, eq. dubiner_functions],
 *    corrected to an orthonormal polynomial basis: the middle factor carries
 *    (1-x)^j and the last Jacobi weight is (2i+2j+2, 0)).
 *  - PML auxiliaries p, q use the same covariant expansion as e, h.
 *  - Mixed orders (mdg_options.mixed = 1): e and p carry N = dim P_{p+1}
 *    modes, h and q carry NH = dim P_p modes, so every H/Q array below is
 *    [nt][3][NH]. The P_p modes are the first NH modes of P_{p+1} (total
 *    degree first), which the library uses to run the mixed system as the
 *    order-(p+1) system with the modes NH.. of h held at zero.
 *  - All host arrays are row-major, caller-owned and only read (or written)
 *    during the call. Device memory is owned by the caller (see
 *    mdg_bind_workspace) or, if the caller passes NULL there, by the library.
 *  - "Synchronous" calls that write device memory (mdg_set_state,
 *    mdg_set_sip_state, mdg_project, mdg_rhs, mdg_rhs_sip, mdg_bind_workspace
 *    on a bound handle) first wait for all work already queued on the device,
 *    on any stream, so they never overwrite data that earlier asynchronous
 *    steps still read.
 *  - Every function returns an mdg_status; on error, mdg_last_error() gives a
 *    message valid until the next call on the same handle. No C++ exception
 *    crosses this boundary. A handle is not thread-safe; use one per stream.
 */
#ifndef MDG_H
#define MDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdg_solver mdg_solver;
typedef int32_t mdg_status;

enum {
  MDG_OK = 0,
  MDG_E_ARG = -1,         /* invalid argument (NULL, size, range) */
  MDG_E_MESH = -2,        /* degenerate/non-manifold/non-finite mesh */
  MDG_E_HIP = -3,         /* HIP runtime error (message has the HIP error) */
  MDG_E_OOM = -4,         /* workspace too small / allocation failed */
  MDG_E_STATE = -5,       /* call order violated (e.g. step before set_mesh) */
  MDG_E_UNSTABLE = -6,    /* energy became non-finite, or grew (mdg_options.monitor) */
  MDG_E_UNSUPPORTED = -7  /* option not compiled in (e.g. order > 4) */
};

enum { MDG_FP64 = 0, MDG_FP32 = 1 };
enum { MDG_CENTRAL = 0, MDG_UPWIND = 1 };
enum { MDG_RK4 = 0, MDG_LEAPFROG = 1 };

typedef struct mdg_options {
  int32_t order;      /* polynomial order p, 1..4 (of h; of e too unless mixed) */
  int32_t precision;  /* MDG_FP64 or MDG_FP32: storage and arithmetic of the state */
  int32_t flux;       /* MDG_CENTRAL [KS eqs. uwc/cwc] or MDG_UPWIND (Riemann flux) */
  int32_t integrator; /* MDG_RK4, or MDG_LEAPFROG (central flux only; see mdg_step) */
  double dt;          /* > 0: fixed time step; 0: computed from cfl */
  double cfl;         /* dt = cfl * min_T(2 r_in,T sqrt(eps_T mu_T)) / (p+1)^2 when dt == 0 */
  int32_t tile;       /* elements per stage-kernel workgroup: 32 or 64; 0 = automatic */
  int32_t mixed;      /* 0: e and h at order p; 1: e at order p+1, h at order p, the paper's
                         pairing [KS eqs. triale, trialh] (then p <= 3) */
  double sip_alpha;   /* > 0: symmetric interior penalty surface unknown h_s on every face
                         [KS Sec. III, eqs. jmp_var_def, 1st_weak_equation, weak_penalty]
                         with alpha_F = sip_alpha (p+1)(p+3)/3 |F| / min(|T|, |T'|), p the
                         order of e;
                         0: none. Central flux only (see mdg_set_sip_state) */
  int32_t monitor;    /* > 0: mdg_step evaluates the FP64 energy of the state every `monitor`
                         steps (and at its start) and returns MDG_E_UNSTABLE when it is not
                         finite or, with RK4 on a mesh without sources, PML elements or the
                         SIP unknown, when it grows by more than a relative 1e-10 (FP64) /
                         1e-5 (FP32) from one check to the next. The semi-discrete energy is conserved by the central flux
                         and decays with the upwind flux [KS Sec. III]; RK4 is strongly stable
                         over two steps, not one, so `monitor` must be >= 2 (MDG_E_ARG). With a
                         monitor mdg_step synchronises its stream before returning. 0: off */
  int32_t mfma;       /* 1: the volume term (the reference-curl contraction of [KS Sec. III,
                         eq. matrix_free_curl]) on the matrix cores, as BF16x3 split products
                         (v_mfma_f32_16x16x32_bf16, each operand split exactly into three
                         bfloat16 parts, six products accumulated in FP32: FP32 accuracy).
                         Needs MDG_FP32, MDG_RK4, order <= 3 and 64-element tiles
                         (MDG_E_UNSUPPORTED otherwise). 0: sparse VALU contraction (default) */
  int32_t launch;     /* stage-kernel grid: MDG_LAUNCH_PERSISTENT, only the workgroups the GPU
                         holds at once, each looping over its tiles and requesting the next
                         tile's input field and halo traces before publishing the current
                         tile's traces (FP32, orders 1-3; one workgroup per tile otherwise);
                         MDG_LAUNCH_PER_TILE, one workgroup per tile, which the hardware
                         dispatches as others finish; MDG_LAUNCH_AUTO (0) = per tile. Results
                         are identical bit for bit */
} mdg_options;

enum { MDG_LAUNCH_AUTO = 0, MDG_LAUNCH_PERSISTENT = 1, MDG_LAUNCH_PER_TILE = 2 };

typedef struct mdg_info {
  int32_t order, nmodes, nfacemodes, precision, flux, tile_size;
  int64_t n_elements, n_faces_interior, n_faces_boundary, n_pml;
  int64_t n_tiles, n_halo;        /* work decomposition of the stage kernel */
  double dt, time;
  double bytes_per_stage;         /* algorithmic HBM bytes of one RK stage, or of one
                                     leap-frog half step (all elements) */
  double flops_per_stage;         /* algorithmic flops of one RK stage (sparse reference ops) */
  int64_t workspace_bytes;        /* device bytes mdg_bind_workspace needs */
  int64_t n_instances;            /* independent instances (mdg_set_instances), >= 1 */
  int64_t n_dipoles;
  int32_t order_h, nmodes_h;      /* order and modes of h (order, nmodes refer to e) */
} mdg_info;

/* Create a solver. opts is copied. *out receives the handle (NULL on error). */
mdg_status mdg_create(const mdg_options* opts, mdg_solver** out);

/* Destroy a handle; frees library-owned device memory. NULL is ignored. */
void mdg_destroy(mdg_solver* s);

/* Message of the last failed call on s (or of the last failed mdg_create when
 * s is NULL). Never NULL. */
const char* mdg_last_error(const mdg_solver* s);

/* Mesh [KS Sec. II]: nv vertices xyz[nv][3], nt tetrahedra tet[nt][4] (vertex
 * ids, any order inside a row). Copies its inputs. Faces with one element are
 * PEC boundary faces [KS Sec. IV]. Errors: MDG_E_MESH for non-finite
 * coordinates, zero-volume tets, repeated vertices or a face shared by more
 * than two tets; MDG_E_ARG for ids out of range. Resets material, PML,
 * sources and state. Host-only (no device call). */
mdg_status mdg_set_mesh(mdg_solver* s, int64_t nv, const double* xyz, int64_t nt,
                        const int64_t* tet);

/* Piecewise-constant material per element [KS Sec. I, constitutive law]:
 * eps[nt], mu[nt] > 0 and finite; NULL means 1. Host-only. */
mdg_status mdg_set_material(mdg_solver* s, const double* eps, const double* mu);

/* PML damping [KS Sec. IV]: omega[nt][3] >= 0, the per-axis damping w_x, w_y,
 * w_z of each element (constant per element, as in [KS Sec. V]). Elements with
 * any w_a > 0 carry the auxiliary fields p, q with eta_a = w_b + w_c - w_a,
 * xi_a = (w_a - w_b)(w_a - w_c) and pole w_a for component a
 * [KS Sec. IV, eqs. p_variable, q_variable]. NULL removes the PML. Host-only. */
mdg_status mdg_set_pml(mdg_solver* s, const double* omega);

/* Point current dipoles j = d delta(r - r0) g(t) [KS Sec. I, current j]:
 * pos[n][3], dir[n][3], wave[n][3] = (f0, bw, t0) with
 * g(t) = sin(2 pi f0 (t - t0)) exp(-(t - t0)^2 / (2 s^2)), s = 1/(2 pi bw).
 * Each dipole acts on the lowest-index element whose closure contains r0
 * (searching the whole mesh). Any n >= 0; n = 0 removes all dipoles. MDG_E_ARG
 * if a point is outside the mesh. Host-only. */
mdg_status mdg_set_dipoles(mdg_solver* s, int32_t n, const double* pos, const double* dir,
                           const double* wave);

/* Independent instances in one solver (many sources or material samples on
 * meshes of uneven size advanced by the same launches): the mesh given to
 * mdg_set_mesh is the disjoint union of n instances whose elements occupy the
 * caller's index ranges [first[i], first[i+1]), first[0] = 0, first[n] = nt.
 * No face may join two instances (MDG_E_MESH). The stage kernel keeps each
 * instance's elements together; all instances share dt (the smallest CFL
 * step when dt is computed). n = 1 with first = {0, nt} is the default.
 * Host-only; call after mdg_set_mesh, before mdg_bind_workspace. */
mdg_status mdg_set_instances(mdg_solver* s, int32_t n, const int64_t* first);

/* Dipoles as in mdg_set_dipoles, dipole i located inside instance inst[i]
 * only (lowest-index element of that instance whose closure contains r0);
 * inst[i] = -1 searches the whole mesh. Host-only. */
mdg_status mdg_set_instance_dipoles(mdg_solver* s, int32_t n, const int32_t* inst, const double* pos,
                                    const double* dir, const double* wave);

/* Device bytes needed by the current setup (finalises the setup: element
 * reordering, tiles, face connectivity). */
mdg_status mdg_workspace_size(mdg_solver* s, size_t* bytes);

/* Bind device memory: dev_ptr must point to >= mdg_workspace_size bytes of
 * device memory on the current HIP device, 256-byte aligned, and outlive the
 * handle (or the next bind). dev_ptr == NULL makes the library allocate it.
 * Uploads the static data on `stream` (a hipStream_t, NULL = default stream)
 * and synchronises that stream. Zeroes the state. MDG_E_UNSUPPORTED if the
 * stage kernel's LDS face-trace exchange (tile size x face modes) exceeds the
 * device's LDS per workgroup (160 KiB on gfx950; only p = 4 in FP64 needs
 * more than 64 KiB). */
mdg_status mdg_bind_workspace(mdg_solver* s, void* dev_ptr, size_t bytes, void* stream);

/* Set the state from host FP64 arrays E[nt][3][N], H[nt][3][N] (covariant
 * coefficients, caller's element order) and PML auxiliaries P, Q (same layout;
 * NULL = zero; ignored on non-PML elements); t is the time of the state.
 * With MDG_LEAPFROG the state is staggered: E and P are taken at t, H and Q
 * at t + dt/2 (mdg_get_state and mdg_project likewise). Synchronous. */
mdg_status mdg_set_state(mdg_solver* s, const double* E, const double* H, const double* P,
                         const double* Q, double t);

/* Copy the state back to host FP64 arrays (same layout; P, Q may be NULL;
 * zero on non-PML elements). Synchronises the device. *t may be NULL. */
mdg_status mdg_get_state(mdg_solver* s, double* E, double* H, double* P, double* Q, double* t);

/* SIP surface unknown (mdg_options.sip_alpha > 0) [KS Sec. III]. On every face
 * F a tangential field h_s of degree p evolves by
 *   (mu_F/alpha_F) (d_t h_s, psi)_F = ([[e]], psi)_F,
 *   [[e]] = n_T x (e_T - e_T') (either side T; n_T x e_T on PEC faces),
 * and adds -(h_s x n_T, v)_F to the E equation of both elements of F
 * [KS eqs. jmp_var_def, 1st_weak_equation, weak_penalty], with
 * mu_F = (mu_T + mu_T')/2 (mu_T on PEC faces), no PML damping of h_s. The
 * block system is then skew and W + 1/2 sum_F (mu_F/alpha_F) (h_s, h_s)_F is
 * conserved by the semi-discrete system (mdg_energy reports W alone). With
 * MDG_LEAPFROG h_s is staggered with h (at t + dt/2). dt from cfl does not
 * account for the penalty: choose cfl (or dt) for it.
 * h_s has the order p of h (also with mixed orders, the paper's pairing).
 * Layout S[nt][4][2][NF] (caller's element order, NF = (p+1)(p+2)/2): face f
 * of element t is the face opposite the element's f-th vertex in the element
 * frame (vertices by ascending global id); its vertices a < b < c (global id)
 * parametrise it as x = x_a + s1 (x_b - x_a) + s2 (x_c - x_a), and
 *   (h_s . t_k)(s) = sum_m S[t][f][k][m] psi_m(s1, s2),  t_1 = x_b - x_a, t_2 = x_c - x_a,
 *   psi_ij = sqrt(2 (2i+1)(i+j+1)) P_i^(0,0)(2 s2/(1-s1) - 1) (1-s1)^i P_j^(2i+1,0)(2 s1 - 1),
 * modes by total degree i+j, then i. Both elements of a face hold a copy; the
 * library updates both from the same data, so they agree to round-off.
 * mdg_set_state and mdg_project set h_s to zero; mdg_set_sip_state then sets
 * it (both copies of a face should be equal). Not available (MDG_E_UNSUPPORTED)
 * with the upwind flux (mdg_create) and in mdg_rhs (see mdg_rhs_sip); the
 * state calls return it without sip_alpha. The probe-energy and adjoint
 * calls carry h_s along (the adjoint negates its skew couplings like the
 * others). Synchronous. */
mdg_status mdg_set_sip_state(mdg_solver* s, const double* S);
mdg_status mdg_get_sip_state(mdg_solver* s, double* S);

/* mdg_rhs with the SIP unknown (mdg_options.sip_alpha > 0): time derivatives
 * (dE, dH, dS, dP, dQ) of the state (E, H, S, P, Q) at time t, S and dS in
 * the layout of mdg_set_sip_state [KS Sec. III, eqs. 1st_weak_equation,
 * weak_penalty]. S == NULL means zero; dS, P, Q, dP, dQ may be NULL. The
 * solver state is not modified (stage scratch is). MDG_E_UNSUPPORTED without
 * sip_alpha (use mdg_rhs). Synchronous. */
mdg_status mdg_rhs_sip(mdg_solver* s, const double* E, const double* H, const double* S, const double* P,
                       const double* Q, double t, double* dE, double* dH, double* dS, double* dP, double* dQ);

/* Physical points where a field must be sampled for mdg_project: q^3 points
 * per element (collapsed Gauss-Legendre rule of order q, 1 <= q <= 16).
 * xyz == NULL: only *npts_per_elem is written. Else xyz[nt][q^3][3]. Host-only. */
mdg_status mdg_projection_points(mdg_solver* s, int32_t q, int64_t* npts_per_elem, double* xyz);

/* L2-project fields sampled at the mdg_projection_points(q) into the state
 * (E = Evals[nt][q^3][3], H = Hvals likewise, Cartesian components; NULL =
 * zero field), auxiliaries zero, time t. Synchronous. */
mdg_status mdg_project(mdg_solver* s, int32_t q, const double* Evals, const double* Hvals,
                       double t);

/* Advance nsteps classic RK4 steps. Asynchronous on `stream` (hipStream_t,
 * NULL = default stream): four stage-kernel launches per step (eight with
 * PML elements, plus a tiny amplitude kernel per stage when dipoles exist).
 * Source amplitudes are evaluated on the device from a device-side clock
 * (t0 + n dt) that the last launch of each step advances, so every launch of
 * a step has the same arguments. Kernel faults surface at the next synchronising call. */
mdg_status mdg_step(mdg_solver* s, int64_t nsteps, void* stream);
/* With MDG_LEAPFROG a step is the staggered leap-frog scheme of [KS Sec. V]
 * instead: e^{n+1} = e^n + dt eps^-1 (curl-terms of h^{n+1/2} - j(t^{n+1/2})),
 * then h^{n+3/2} = h^{n+1/2} - dt mu^-1 (curl-terms of e^{n+1}), one launch
 * per half step (two with PML elements), each updating its field in place.
 * The PML damping terms are taken by the trapezoid rule, which keeps the
 * scheme explicit (a 2x2 solve per Cartesian component) [KS Sec. V]. Needs
 * the central flux: without PML the staggered energy
 * 1/2 (e^n, eps e^n) + 1/2 (h^{n-1/2}, mu h^{n+1/2}) is then conserved to
 * round-off; stable for dt rho(L) < 2 (a smaller CFL number than RK4's). */

/* Same result as mdg_step(nsteps), launched as replays of a HIP graph of
 * steps_per_graph steps (captured on the first call, kept until the solver
 * is re-bound or destroyed; remainder steps run eagerly). `stream` must be a
 * non-default hipStream_t (capture needs one); MDG_E_ARG otherwise. */
mdg_status mdg_step_graph(mdg_solver* s, int64_t nsteps, int32_t steps_per_graph, void* stream);

/* One operator application [KS Sec. III-IV]: time derivatives (dE, dH, dP, dQ)
 * of the given state at time t (source evaluated at t), same layouts as
 * mdg_set_state. The solver state is not modified (stage scratch is).
 * Synchronous. dP/dQ/P/Q may be NULL. */
mdg_status mdg_rhs(mdg_solver* s, const double* E, const double* H, const double* P,
                   const double* Q, double t, double* dE, double* dH, double* dP, double* dQ);

/* Probe energy alone: advances nsteps steps (RK4 or leap-frog) from the
 * current state accumulating on the device
 *   J = sum_{n=1..nsteps} dt sum_{T in probes} ||e^n||^2_{L2(T)}
 * (the objective of mdg_adjoint_probe_energy; element indices probes[nprobe]
 * in the caller's order), written to *J. The solver ends in the advanced
 * state. Synchronous. */
mdg_status mdg_probe_energy(mdg_solver* s, int64_t nsteps, int32_t nprobe, const int64_t* probes, double* J,
                            void* stream);

/* Same as mdg_probe_energy, allocating no device memory, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The accumulator and the probe list live in
 * a library-wide device array of 256 + 8 MDG_NOALLOC_MAX_PROBES bytes, one copy
 * per GPU, held until the process ends and set up on the first call on each
 * device. nprobe > MDG_NOALLOC_MAX_PROBES gives MDG_E_ARG. The accumulator is
 * cleared at the start of every call; calls that overlap on one GPU (handles
 * driven from several host threads or streams at once) race on that array
 * and must be serialised by the caller. Synchronous. */
#define MDG_NOALLOC_MAX_PROBES 4096
mdg_status mdg_probe_energy_noalloc(mdg_solver* s, int64_t nsteps, int32_t nprobe, const int64_t* probes,
                                    double* J, void* stream);

/* Probe energy and its gradient with respect to every element's permittivity
 * (the material of [KS Sec. I]), by the discrete adjoint of the RK4 steps.
 * From the current state, advances nsteps steps (the solver ends in the
 * advanced state) accumulating
 *   J = sum_{n=1..nsteps} dt sum_{T in probes} ||e^n||^2_{L2(T)},
 * then sweeps the adjoint of every step backwards, recomputing the forward
 * states and stage derivatives of each interval of `every` steps from
 * checkpoints kept on the device, and returns J and grad_eps[nt] = dJ/deps_T (caller's element order;
 * FP64 reductions, the state precision of the solver). probes[nprobe] are
 * element indices. Requires MDG_RK4 (MDG_E_UNSUPPORTED). The averaged part
 * of the face terms and the volume curl are skew, the upwind penalties
 * symmetric, so the adjoint operator in the mass inner product is the forward
 * one with the skew part negated and the PML couplings of [KS Sec. IV]
 * transposed. eps enters through the mass inverse of the curl part (the PML
 * equations are written for P/eps and Q/mu, whose values at the start are
 * held fixed: zero for a PML at rest) and, with the upwind flux, through the
 * face impedances sqrt(mu/eps) of every face of an element.
 * Allocates (ceil(nsteps/every) + 5 min(every, nsteps) + 6) state vectors
 * (fields, PML auxiliaries, SIP unknown) of device memory for the call
 * (MDG_E_OOM if they do not fit: a smaller `every` needs less). Synchronous. */
mdg_status mdg_adjoint_probe_energy(mdg_solver* s, int64_t nsteps, int32_t every, int32_t nprobe,
                                     const int64_t* probes, double* J, double* grad_eps, void* stream);

/* Electromagnetic energy W = 1/2 sum_T [(eps e, e)_T + (mu h, h)_T] of the
 * current state, accumulated in FP64 on the device [KS Sec. III]. Synchronous. */
mdg_status mdg_energy(mdg_solver* s, double* W);

/* Energy of each instance, W[n_instances], FP64 per-element values summed in
 * element order on the host. Synchronous. */
mdg_status mdg_energy_instances(mdg_solver* s, double* W);

/* Sizes, decomposition and algorithmic cost of the current setup. */
mdg_status mdg_query(mdg_solver* s, mdg_info* info);

#ifdef __cplusplus
}
#endif
#endif /* MDG_H */

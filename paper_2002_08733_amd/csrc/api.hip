// api.hip -- extern "C" entry points of libmdg (declared in include/mdg.h).
//
// Host-only calls (mesh, material, PML, dipoles, projection points, query)
// never touch the device. Device memory is either bound by the caller or
// allocated here on demand; all device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "refbasis.hpp"
#include "solver.hpp"

using namespace mdg;

struct mdg_solver {
  Solver s;
};

namespace {

thread_local std::string g_create_error;

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
mdg_status guarded(mdg_solver* h, F&& fn) {
  if (!h) return MDG_E_ARG;
  try {
    h->s.err.clear();
    fn(h->s);
    return MDG_OK;
  } catch (const Error& e) {
    h->s.err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->s.err = "host allocation failed";
    return MDG_E_OOM;
  } catch (const std::exception& e) {
    h->s.err = e.what();
    return MDG_E_ARG;
  }
}

void need_mesh(const Solver& s) {
  if (s.nt == 0) throw Error(MDG_E_STATE, "no mesh: call mdg_set_mesh first");
}

void need_bound(const Solver& s) {
  need_mesh(s);
  if (!s.bound) throw Error(MDG_E_STATE, "no workspace: call mdg_bind_workspace after the setup calls");
}

char* dev(const Solver& s, size_t off) { return static_cast<char*>(s.ws) + off; }

// The synchronous calls that write device memory (state, SIP unknown, clock,
// operator input) upload on the NULL stream, which a non-blocking caller
// stream (e.g. the one mdg_step_graph needs) does not order against: wait
// for all work queued so far on the device before writing.
void quiesce() { hip_check(hipDeviceSynchronize(), "synchronize before a host write"); }

// host FP64 SoA rows -> device array of the solver's precision
void upload(const Solver& s, const std::vector<double>& h, size_t off, hipStream_t st) {
  if (h.empty()) return;
  if (s.opt.precision == MDG_FP32) {
    std::vector<float> f(h.begin(), h.end());
    hip_check(hipMemcpyAsync(dev(s, off), f.data(), f.size() * 4, hipMemcpyHostToDevice, st), "upload");
    hip_check(hipStreamSynchronize(st), "upload sync");
  } else {
    hip_check(hipMemcpyAsync(dev(s, off), h.data(), h.size() * 8, hipMemcpyHostToDevice, st), "upload");
    hip_check(hipStreamSynchronize(st), "upload sync");
  }
}

void download(const Solver& s, size_t off, size_t n, std::vector<double>& h) {
  h.resize(n);
  if (s.opt.precision == MDG_FP32) {
    std::vector<float> f(n);
    hip_check(hipMemcpy(f.data(), dev(s, off), n * 4, hipMemcpyDeviceToHost), "download");
    for (size_t i = 0; i < n; ++i) h[i] = f[i];
  } else {
    hip_check(hipMemcpy(h.data(), dev(s, off), n * 8, hipMemcpyDeviceToHost), "download");
  }
}

void ensure_final(Solver& s) {
  need_mesh(s);
  if (!s.finalized) finalize(s);
}

void write_state(Solver& s, const double* E, const double* H, const double* P, const double* Q, size_t off,
                 size_t aoff) {
  quiesce();
  std::vector<double> buf;
  pack_state(s, E, H, buf);
  upload(s, buf, off, nullptr);
  if (s.Kp > 0) {
    pack_aux(s, P, Q, buf);
    upload(s, buf, aoff, nullptr);
  }
}

void read_state(Solver& s, double* E, double* H, double* P, double* Q, size_t off, size_t aoff) {
  hip_check(hipDeviceSynchronize(), "synchronize");
  std::vector<double> buf;
  if (E || H) {
    download(s, off, size_t(state_rows(s)) * s.Kpad, buf);
    unpack_state(s, buf, E, H);
  }
  if (P || Q) {
    if (s.Kp > 0) {
      download(s, aoff, size_t(state_rows(s)) * s.Kppad, buf);
      unpack_aux(s, buf, P, Q);
    } else {
      if (P) std::memset(P, 0, size_t(s.nt) * 3 * s.N * sizeof(double));
      if (Q) std::memset(Q, 0, size_t(s.nt) * 3 * s.NH * sizeof(double));
    }
  }
}

// a new state starts with a zero SIP unknown
void clear_sip(Solver& s) {
  if (!s.sip()) return;
  quiesce();
  std::vector<double> z;
  pack_sip(s, nullptr, z);
  upload(s, z, s.L.sY, nullptr);
}

void no_sip(const Solver& s, const char* what) {
  if (s.sip()) throw Error(MDG_E_UNSUPPORTED, std::string(what) + ": not available with the SIP unknown");
}

// set a device clock (t0, n); synchronous
void set_clock(Solver& s, size_t off, double t0, double n = 0.0) {
  const double c[2] = {t0, n};
  quiesce();
  hip_check(hipMemcpy(dev(s, off), c, sizeof c, hipMemcpyHostToDevice), "clock");
}

// device buffers owned by one call, freed on every exit path
struct DevBufs {
  std::vector<void*> p;
  void* get(size_t bytes) {
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) throw Error(MDG_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    p.push_back(q);
    return q;
  }
  ~DevBufs() {
    for (void* q : p) (void)hipFree(q);
  }
};

void drop_graph(Solver& s) {
  if (s.graph_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(s.graph_exec));
  if (s.graph) (void)hipGraphDestroy(static_cast<hipGraph_t>(s.graph));
  s.graph_exec = nullptr;
  s.graph = nullptr;
  s.graph_steps = 0;
}

// n leap-frog steps: the E half (sources at t + dt/2), then the H half, which
// advances the clock; both update Y (and the PML auxiliaries) in place and
// share the halo buffer H0
void enqueue_leapfrog_steps(Solver& s, int64_t nsteps, void* stream) {
  const DevLayout& L = s.L;
  for (int64_t n = 0; n < nsteps; ++n) {
    for (int half = 0; half < 2; ++half) {
      StageParams sp{};
      sp.stage = 4 + half;
      sp.dt = s.dt;
      sp.cstage = 0.5;
      sp.clock = reinterpret_cast<const double*>(dev(s, L.clock));
      sp.sources = half == 0;
      sp.Y = dev(s, L.Y);
      sp.Uin = sp.Y;
      sp.Uout = sp.Y;
      sp.ACC = dev(s, L.ACC);
      sp.aY = dev(s, L.aY);
      sp.aUin = sp.aY;
      sp.aUout = sp.aY;
      sp.aACC = dev(s, L.aACC);
      sp.sY = dev(s, L.sY);
      sp.sUin = sp.sY;
      sp.sUout = sp.sY;
      sp.sACC = dev(s, L.sACC);
      sp.hin = dev(s, L.H0);
      sp.hout = dev(s, L.H0);
      sp.publish = true;
      if (half == 1) sp.tick = reinterpret_cast<double*>(dev(s, L.clock));
      launch_stage(s, sp, stream);
    }
  }
}

// the arrays of one RK4 stepping: base Y, stage inputs Ua/Ub, accumulator
// ACC, for the fields (E, H), the PML auxiliaries and the SIP unknown
struct RKBufs {
  void *Y, *Ua, *Ub, *ACC;
  void *aY, *aUa, *aUb, *aACC;
  void *sY, *sUa, *sUb, *sACC;
  // optional: the new state goes to Yout instead of Y; stage i stores its
  // derivative in K[i]
  void *Yout = nullptr, *aYout = nullptr, *sYout = nullptr;
  void *K[4] = {}, *aK[4] = {}, *sK[4] = {};
};

RKBufs solver_bufs(const Solver& s) {
  const DevLayout& L = s.L;
  return RKBufs{dev(s, L.Y),  dev(s, L.Ua),  dev(s, L.Ub),  dev(s, L.ACC), dev(s, L.aY),  dev(s, L.aUa),
                dev(s, L.aUb), dev(s, L.aACC), dev(s, L.sY), dev(s, L.sUa), dev(s, L.sUb), dev(s, L.sACC)};
}

static const double RK_B[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
static const double RK_C[4] = {0.0, 0.5, 0.5, 1.0};

// one classic RK4 step of the arrays b, one stage launch each (two with PML
// elements): stage inputs Y -> Ua -> Ub -> Ua, the final update in place
// into Y (or into b.Yout). The halo traces of Y must be in H0 (those of the
// new state are there after the step).
// adj: the adjoint operator in the mass inner product (no sources); tick:
// clock advanced by the last launch, or null. before(i, in): called before
// stage i is enqueued, with the arrays of its input (Y, Ua or Ub).
template <typename F>
void enqueue_rk4_step(Solver& s, const RKBufs& b, const double* clock, bool sources, bool adj, double* tick,
                      void* stream, F&& before) {
  const DevLayout& L = s.L;
  for (int i = 0; i < 4; ++i) {
    StageParams sp{};
    sp.stage = i;
    sp.bcoef = RK_B[i];
    sp.cdt = i < 3 ? RK_C[i + 1] * s.dt : 0.0;
    sp.dt = s.dt;
    sp.cstage = RK_C[i];
    sp.clock = clock;
    sp.sources = sources;
    sp.adj = adj;
    const int in = i == 0 ? 0 : (i == 2 ? 2 : 1);  // Y, Ua, Ub
    void* const U[3] = {b.Y, b.Ua, b.Ub};
    void* const aU[3] = {b.aY, b.aUa, b.aUb};
    void* const sU[3] = {b.sY, b.sUa, b.sUb};
    before(i, U[in], aU[in], sU[in]);
    sp.Y = b.Y;
    sp.Uin = U[in];
    sp.Uout = i == 1 ? b.Ub : b.Ua;
    sp.ACC = b.ACC;
    sp.aY = b.aY;
    sp.aUin = aU[in];
    sp.aUout = i == 1 ? b.aUb : b.aUa;
    sp.aACC = b.aACC;
    sp.sY = b.sY;
    sp.sUin = sU[in];
    sp.sUout = i == 1 ? b.sUb : b.sUa;
    sp.sACC = b.sACC;
    sp.Yout = b.Yout;
    sp.aYout = b.aYout;
    sp.sYout = b.sYout;
    sp.Kout = b.K[i];
    sp.aKout = b.aK[i];
    sp.sKout = b.sK[i];
    // halo traces of the stage input in, of the stage output out
    sp.hin = dev(s, (i & 1) ? L.H1 : L.H0);
    sp.hout = dev(s, (i & 1) ? L.H0 : L.H1);
    sp.publish = true;
    if (i == 3) sp.tick = tick;
    launch_stage(s, sp, stream);
  }
}

// enqueue n steps: RK4 (4 or 8 stage launches each; the last advances the
// clock) or leap-frog
void enqueue_steps(Solver& s, int64_t nsteps, void* stream) {
  if (s.opt.integrator == MDG_LEAPFROG) {
    enqueue_leapfrog_steps(s, nsteps, stream);
    return;
  }
  const RKBufs b = solver_bufs(s);
  double* clock = reinterpret_cast<double*>(dev(s, s.L.clock));
  for (int64_t n = 0; n < nsteps; ++n)
    enqueue_rk4_step(s, b, clock, true, false, clock, stream, [](int, const void*, const void*, const void*) {});
}

void publish_if_needed(Solver& s, void* stream) {
  if (!s.halo_valid) {
    launch_publish(s, dev(s, s.L.Y), dev(s, s.L.H0), stream);
    s.halo_valid = true;
  }
}

// one operator application from host arrays (the SIP unknown from S, zero
// when null); the input's halo traces go to H1, so H0 keeps those of Y
void host_rhs(Solver& s, const double* E, const double* H, const double* S, const double* P, const double* Q,
              double t, double* dE, double* dH, double* dS, double* dP, double* dQ) {
  need_bound(s);
  if (!E || !H || !dE || !dH) throw Error(MDG_E_ARG, "E, H, dE, dH are required");
  quiesce();
  const DevLayout& L = s.L;
  write_state(s, E, H, P, Q, L.Ua, L.aUa);
  if (s.sip()) {
    std::vector<double> buf;
    pack_sip(s, S, buf);
    upload(s, buf, L.sUa, nullptr);
  }
  StageParams sp{};
  sp.stage = -1;
  sp.dt = s.dt;
  sp.cstage = 0.0;
  set_clock(s, L.rhs_clock, t);
  sp.clock = reinterpret_cast<const double*>(dev(s, L.rhs_clock));
  sp.Y = dev(s, L.Y);
  sp.Uin = dev(s, L.Ua);
  sp.Uout = dev(s, L.Ub);
  sp.ACC = dev(s, L.ACC);
  sp.aY = dev(s, L.aY);
  sp.aUin = dev(s, L.aUa);
  sp.aUout = dev(s, L.aUb);
  sp.aACC = dev(s, L.aACC);
  sp.sY = dev(s, L.sY);
  sp.sUin = dev(s, L.sUa);
  sp.sUout = dev(s, L.sUb);
  sp.sACC = dev(s, L.sACC);
  launch_publish(s, dev(s, L.Ua), dev(s, L.H1), nullptr);
  sp.hin = dev(s, L.H1);
  sp.hout = nullptr;
  sp.publish = false;
  launch_stage(s, sp, nullptr);
  read_state(s, dE, dH, dP, dQ, L.Ub, L.aUb);
  if (s.sip() && dS) {
    std::vector<double> buf;
    download(s, L.sUb, size_t(8) * s.NF * s.Kpad, buf);
    unpack_sip(s, buf, dS);
  }
}

}  // namespace

// ------------------------------------------------ allocation-free probe energy
// For callers that cannot allocate device memory: the accumulator (bytes
// 0..7) and the probe list (from byte 256, int64) of mdg_probe_energy_noalloc
// live in this array, one copy per GPU, held until the process ends. In host
// code `scratch` names a host-side stand-in: kernels and copies get the
// device address from hipGetSymbolAddress, kept per device.
static __device__ __align__(256) unsigned char scratch[256 + 8 * MDG_NOALLOC_MAX_PROBES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// device address of `scratch` on the current device (looked up once per device)
unsigned char* scratch_ptr() {
  int d = 0;
  hip_check(hipGetDevice(&d), "hipGetDevice");
  if (d < 0 || d >= MAX_DEVICES) throw Error(MDG_E_HIP, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[d]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Error(MDG_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[d] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[d]);
}

// clears the accumulator with a kernel (no memset node if the caller captures)
__global__ void zero_one(double* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0.0;
}

}  // namespace

extern "C" {

mdg_status mdg_create(const mdg_options* o, mdg_solver** out) {
  if (!out) return MDG_E_ARG;
  *out = nullptr;
  g_create_error.clear();
  if (!o) { g_create_error = "NULL options"; return MDG_E_ARG; }
  if (o->mixed != 0 && o->mixed != 1) { g_create_error = "mixed must be 0 or 1"; return MDG_E_ARG; }
  if (o->order < 1 || o->order + o->mixed > 4) {
    g_create_error = "order must be 1..4 (1..3 with mixed orders)";
    return MDG_E_UNSUPPORTED;
  }
  if (o->precision != MDG_FP64 && o->precision != MDG_FP32) { g_create_error = "bad precision"; return MDG_E_ARG; }
  if (o->flux != MDG_CENTRAL && o->flux != MDG_UPWIND) { g_create_error = "bad flux"; return MDG_E_ARG; }
  if (o->integrator != MDG_RK4 && o->integrator != MDG_LEAPFROG) { g_create_error = "bad integrator"; return MDG_E_ARG; }
  if (o->integrator == MDG_LEAPFROG && o->flux != MDG_CENTRAL) {
    g_create_error = "leap-frog needs the central flux";
    return MDG_E_UNSUPPORTED;
  }
  if (o->tile != 0 && o->tile != 32 && o->tile != 64) { g_create_error = "tile must be 0, 32 or 64"; return MDG_E_ARG; }
  if (!(o->sip_alpha >= 0) || !std::isfinite(o->sip_alpha)) { g_create_error = "sip_alpha must be >= 0"; return MDG_E_ARG; }
  if (o->sip_alpha > 0 && o->flux != MDG_CENTRAL) {
    g_create_error = "the SIP unknown needs the central flux";
    return MDG_E_UNSUPPORTED;
  }
  if (!(o->dt >= 0) || (o->dt == 0 && !(o->cfl > 0))) { g_create_error = "need dt > 0 or cfl > 0"; return MDG_E_ARG; }
  if (o->monitor < 0 || o->monitor == 1) { g_create_error = "monitor must be 0 or >= 2"; return MDG_E_ARG; }
  if (o->mfma != 0 && o->mfma != 1) { g_create_error = "mfma must be 0 or 1"; return MDG_E_ARG; }
  if (o->launch < MDG_LAUNCH_AUTO || o->launch > MDG_LAUNCH_PER_TILE) {
    g_create_error = "launch must be MDG_LAUNCH_AUTO, MDG_LAUNCH_PERSISTENT or MDG_LAUNCH_PER_TILE";
    return MDG_E_ARG;
  }
  if (o->mfma && (o->precision != MDG_FP32 || o->integrator != MDG_RK4 || o->order + o->mixed > 3 ||
                  (o->tile != 0 && o->tile != 64))) {
    g_create_error = "the MFMA volume term needs FP32, RK4, order <= 3 and 64-element tiles";
    return MDG_E_UNSUPPORTED;
  }
  mdg_solver* h = new (std::nothrow) mdg_solver();
  if (!h) return MDG_E_OOM;
  h->s.opt = *o;
  h->s.P = o->order + o->mixed;
  h->s.N = nmodes3(h->s.P);
  h->s.NF = nmodes2(h->s.P);
  h->s.NH = nmodes3(o->order);
  h->s.NFH = nmodes2(o->order);
  *out = h;
  return MDG_OK;
}

void mdg_destroy(mdg_solver* h) {
  if (!h) return;
  drop_graph(h->s);
  if (h->s.ws_owned && h->s.ws) (void)hipFree(h->s.ws);
  delete h;
}

const char* mdg_last_error(const mdg_solver* h) {
  if (!h) return g_create_error.c_str();
  return h->s.err.c_str();
}

mdg_status mdg_set_mesh(mdg_solver* h, int64_t nv, const double* xyz, int64_t nt, const int64_t* tet) {
  return guarded(h, [&](Solver& s) { setup_mesh(s, nv, xyz, nt, tet); });
}

mdg_status mdg_set_material(mdg_solver* h, const double* eps, const double* mu) {
  return guarded(h, [&](Solver& s) { need_mesh(s); setup_material(s, eps, mu); });
}

mdg_status mdg_set_pml(mdg_solver* h, const double* omega) {
  return guarded(h, [&](Solver& s) { need_mesh(s); setup_pml(s, omega); });
}

mdg_status mdg_set_dipoles(mdg_solver* h, int32_t n, const double* pos, const double* dir, const double* wave) {
  return guarded(h, [&](Solver& s) { need_mesh(s); setup_dipoles(s, n, nullptr, pos, dir, wave); });
}

mdg_status mdg_set_instances(mdg_solver* h, int32_t n, const int64_t* first) {
  return guarded(h, [&](Solver& s) { need_mesh(s); setup_instances(s, n, first); });
}

mdg_status mdg_set_instance_dipoles(mdg_solver* h, int32_t n, const int32_t* inst, const double* pos,
                                    const double* dir, const double* wave) {
  return guarded(h, [&](Solver& s) {
    need_mesh(s);
    if (n > 0 && !inst) throw Error(MDG_E_ARG, "set_instance_dipoles: NULL inst");
    setup_dipoles(s, n, inst, pos, dir, wave);
  });
}

mdg_status mdg_workspace_size(mdg_solver* h, size_t* bytes) {
  return guarded(h, [&](Solver& s) {
    if (!bytes) throw Error(MDG_E_ARG, "NULL bytes");
    ensure_final(s);
    *bytes = s.L.total;
  });
}

mdg_status mdg_bind_workspace(mdg_solver* h, void* ptr, size_t bytes, void* stream) {
  return guarded(h, [&](Solver& s) {
    ensure_final(s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s.bound) quiesce();  // work queued on the old workspace
    {
      int dev_id = 0, lds_max = 0;
      hip_check(hipGetDevice(&dev_id), "hipGetDevice");
      hip_check(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id),
                "hipDeviceGetAttribute");
      if (stage_lds_bytes(s) > size_t(lds_max))
        throw Error(MDG_E_UNSUPPORTED, "face-trace exchange needs " + std::to_string(stage_lds_bytes(s)) +
                                           " B of LDS, the device allows " + std::to_string(lds_max));
    }
    drop_graph(s);
    if (s.ws_owned && s.ws) {
      hip_check(hipFree(s.ws), "hipFree");
      s.ws = nullptr;
      s.ws_owned = false;
    }
    s.bound = false;
    if (!ptr) {
      void* p = nullptr;
      hipError_t e = hipMalloc(&p, s.L.total);
      if (e != hipSuccess) throw Error(MDG_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
      s.ws = p;
      s.ws_owned = true;
    } else {
      if (bytes < s.L.total) throw Error(MDG_E_OOM, "workspace smaller than mdg_workspace_size");
      if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) throw Error(MDG_E_ARG, "workspace must be 256-byte aligned");
      s.ws = ptr;
    }
    s.ws_bytes = s.L.total;
    hip_check(hipMemsetAsync(s.ws, 0, s.L.total, st), "hipMemsetAsync");
    hip_check(hipStreamSynchronize(st), "sync");
    upload(s, s.geo, s.L.geo, st);
    hip_check(hipMemcpyAsync(dev(s, s.L.nbr), s.nbr_code.data(), s.nbr_code.size() * 4, hipMemcpyHostToDevice, st), "nbr");
    hip_check(hipMemcpyAsync(dev(s, s.L.nbrg), s.nbr_glob.data(), s.nbr_glob.size() * 4, hipMemcpyHostToDevice, st),
              "nbrg");
    hip_check(hipMemcpyAsync(dev(s, s.L.pub), s.pub_code.data(), s.pub_code.size() * 4, hipMemcpyHostToDevice, st), "pub");
    hip_check(hipMemcpyAsync(dev(s, s.L.halo_tile), s.halo_tile.data(), s.halo_tile.size() * 4, hipMemcpyHostToDevice, st), "halo");
    hip_check(hipStreamSynchronize(st), "sync");
    if (s.Kp > 0) upload(s, s.pmlrec, s.L.pml, st);
    if (!s.dips.empty()) {
      // load vectors, waveforms, and for every element the chain of dipoles on it
      const size_t nd = s.dips.size();
      std::vector<double> src(nd * 3 * s.N, 0.0), wave(nd * 3);
      std::vector<int32_t> first(s.Kpad, -1), next(nd, -1);
      for (size_t i = nd; i-- > 0;) {
        std::copy(s.dips[i].coef.begin(), s.dips[i].coef.end(), src.begin() + i * 3 * s.N);
        for (int c = 0; c < 3; ++c) wave[3 * i + c] = s.dips[i].wave[c];
        const int64_t k = s.iperm[s.dips[i].elem];
        next[i] = first[k];
        first[k] = (int32_t)i;
      }
      upload(s, src, s.L.src, st);
      hip_check(hipMemcpyAsync(dev(s, s.L.srcwave), wave.data(), wave.size() * 8, hipMemcpyHostToDevice, st), "src");
      hip_check(hipMemcpyAsync(dev(s, s.L.srcid), first.data(), first.size() * 4, hipMemcpyHostToDevice, st), "src");
      hip_check(hipMemcpyAsync(dev(s, s.L.srcnext), next.data(), next.size() * 4, hipMemcpyHostToDevice, st), "src");
      hip_check(hipStreamSynchronize(st), "sync");
    }
    s.dt = s.opt.dt > 0 ? s.opt.dt : cfl_dt(s);
    s.t0 = 0.0;
    s.nstep = 0;
    set_clock(s, s.L.clock, 0.0);
    s.halo_valid = true;  // zero state, zero traces
    s.bound = true;
  });
}

mdg_status mdg_set_state(mdg_solver* h, const double* E, const double* H, const double* P, const double* Q,
                         double t) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (!E || !H) throw Error(MDG_E_ARG, "E and H are required");
    write_state(s, E, H, P, Q, s.L.Y, s.L.aY);
    clear_sip(s);
    s.halo_valid = false;
    s.t0 = t;
    s.nstep = 0;
    set_clock(s, s.L.clock, t);
  });
}

mdg_status mdg_get_state(mdg_solver* h, double* E, double* H, double* P, double* Q, double* t) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    read_state(s, E, H, P, Q, s.L.Y, s.L.aY);
    if (t) *t = s.time();
  });
}

mdg_status mdg_set_sip_state(mdg_solver* h, const double* S) {
  return guarded(h, [&](Solver& s) {
    if (!s.sip()) throw Error(MDG_E_UNSUPPORTED, "set_sip_state: the solver has no SIP unknown (sip_alpha = 0)");
    need_bound(s);
    if (!S) throw Error(MDG_E_ARG, "set_sip_state: NULL S");
    quiesce();
    std::vector<double> buf;
    pack_sip(s, S, buf);
    upload(s, buf, s.L.sY, nullptr);
  });
}

mdg_status mdg_get_sip_state(mdg_solver* h, double* S) {
  return guarded(h, [&](Solver& s) {
    if (!s.sip()) throw Error(MDG_E_UNSUPPORTED, "get_sip_state: the solver has no SIP unknown (sip_alpha = 0)");
    need_bound(s);
    if (!S) throw Error(MDG_E_ARG, "get_sip_state: NULL S");
    hip_check(hipDeviceSynchronize(), "synchronize");
    std::vector<double> buf;
    download(s, s.L.sY, size_t(8) * s.NF * s.Kpad, buf);
    unpack_sip(s, buf, S);
  });
}

mdg_status mdg_projection_points(mdg_solver* h, int32_t q, int64_t* npts, double* xyz) {
  return guarded(h, [&](Solver& s) {
    need_mesh(s);
    if (q < 1 || q > 16) throw Error(MDG_E_ARG, "q must be 1..16");
    if (npts) *npts = int64_t(q) * q * q;
    if (xyz) projection_points(s, q, xyz);
  });
}

mdg_status mdg_project(mdg_solver* h, int32_t q, const double* Ev, const double* Hv, double t) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (q < 1 || q > 16) throw Error(MDG_E_ARG, "q must be 1..16");
    std::vector<double> ce, ch;
    if (Ev) project_fields(s, q, Ev, s.N, ce); else ce.assign(size_t(s.nt) * 3 * s.N, 0.0);
    if (Hv) project_fields(s, q, Hv, s.NH, ch); else ch.assign(size_t(s.nt) * 3 * s.NH, 0.0);
    write_state(s, ce.data(), ch.data(), nullptr, nullptr, s.L.Y, s.L.aY);
    clear_sip(s);
    s.halo_valid = false;
    s.t0 = t;
    s.nstep = 0;
    set_clock(s, s.L.clock, t);
  });
}

mdg_status mdg_step(mdg_solver* h, int64_t nsteps, void* stream) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (nsteps < 0) throw Error(MDG_E_ARG, "nsteps < 0");
    if (nsteps == 0) return;
    publish_if_needed(s, stream);
    const int64_t k = s.opt.monitor;
    if (k <= 0) {
      enqueue_steps(s, nsteps, stream);
      s.nstep += nsteps;
      return;
    }
    // energy monitor: the energy at the start, then after every k steps (and
    // at the end); growth is a failure only where this energy must not grow:
    // RK4 without sources, PML elements or the SIP unknown (whose face energy
    // the field energy exchanges with)
    const bool growth = s.dips.empty() && s.Kp == 0 && !s.sip() && s.opt.integrator == MDG_RK4;
    const double tol = s.opt.precision == MDG_FP32 ? 1e-5 : 1e-10;
    hipStream_t st = static_cast<hipStream_t>(stream);
    launch_energy(s, dev(s, s.L.Y), stream);
    launch_monitor(s, true, growth, tol, stream);
    for (int64_t done = 0; done < nsteps;) {
      const int64_t n = std::min<int64_t>(k, nsteps - done);
      enqueue_steps(s, n, stream);
      done += n;
      launch_energy(s, dev(s, s.L.Y), stream);
      launch_monitor(s, false, growth, tol, stream);
    }
    s.nstep += nsteps;
    double mon[4];
    hip_check(hipStreamSynchronize(st), "sync");
    hip_check(hipMemcpy(mon, dev(s, s.L.mon), sizeof mon, hipMemcpyDeviceToHost), "monitor");
    if (mon[1] == 2.0) throw Error(MDG_E_UNSTABLE, "energy is not finite");
    if (mon[1] == 1.0)
      throw Error(MDG_E_UNSTABLE, "energy grew between two checks (from " + std::to_string(mon[2]) + " to " +
                                      std::to_string(mon[3]) + " over the call)");
  });
}

mdg_status mdg_step_graph(mdg_solver* h, int64_t nsteps, int32_t steps_per_graph, void* stream) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (nsteps < 0 || steps_per_graph < 1) throw Error(MDG_E_ARG, "nsteps >= 0 and steps_per_graph >= 1");
    if (!stream) throw Error(MDG_E_ARG, "step_graph: graph capture needs a non-default stream");
    if (nsteps == 0) return;
    hipStream_t st = static_cast<hipStream_t>(stream);
    publish_if_needed(s, stream);
    if (s.graph_exec && s.graph_steps != steps_per_graph) drop_graph(s);
    if (!s.graph_exec && nsteps >= steps_per_graph) {
      hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      try {
        enqueue_steps(s, steps_per_graph, stream);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hipGraph_t g = nullptr;
      hip_check(hipStreamEndCapture(st, &g), "hipStreamEndCapture");
      hipGraphExec_t ge = nullptr;
      const hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        hip_check(e, "hipGraphInstantiate");
      }
      s.graph = g;
      s.graph_exec = ge;
      s.graph_steps = steps_per_graph;
    }
    int64_t left = nsteps;
    while (s.graph_exec && left >= s.graph_steps) {
      hip_check(hipGraphLaunch(static_cast<hipGraphExec_t>(s.graph_exec), st), "hipGraphLaunch");
      left -= s.graph_steps;
    }
    if (left > 0) enqueue_steps(s, left, stream);
    s.nstep += nsteps;
  });
}

mdg_status mdg_rhs_sip(mdg_solver* h, const double* E, const double* H, const double* S, const double* P,
                       const double* Q, double t, double* dE, double* dH, double* dS, double* dP, double* dQ) {
  return guarded(h, [&](Solver& s) {
    if (!s.sip()) throw Error(MDG_E_UNSUPPORTED, "rhs_sip: the solver has no SIP unknown (use mdg_rhs)");
    host_rhs(s, E, H, S, P, Q, t, dE, dH, dS, dP, dQ);
  });
}

mdg_status mdg_rhs(mdg_solver* h, const double* E, const double* H, const double* P, const double* Q, double t,
                   double* dE, double* dH, double* dP, double* dQ) {
  return guarded(h, [&](Solver& s) {
    no_sip(s, "rhs (use mdg_rhs_sip)");
    host_rhs(s, E, H, nullptr, P, Q, t, dE, dH, nullptr, dP, dQ);
  });
}

mdg_status mdg_probe_energy(mdg_solver* h, int64_t nsteps, int32_t nprobe, const int64_t* probes, double* J,
                            void* stream) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (nsteps < 0) throw Error(MDG_E_ARG, "probe energy: nsteps >= 0");
    if (nprobe < 1 || !probes || !J) throw Error(MDG_E_ARG, "probe energy: probes and J required");
    std::vector<int64_t> pin(nprobe);
    for (int i = 0; i < nprobe; ++i) {
      if (probes[i] < 0 || probes[i] >= s.nt) throw Error(MDG_E_ARG, "probe energy: element out of range");
      pin[i] = s.iperm[probes[i]];
    }
    DevBufs B;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* Jd = static_cast<double*>(B.get(8));
    int64_t* pd = static_cast<int64_t*>(B.get(size_t(nprobe) * 8));
    hip_check(hipMemcpyAsync(pd, pin.data(), pin.size() * 8, hipMemcpyHostToDevice, st), "probes");
    hip_check(hipMemsetAsync(Jd, 0, 8, st), "J");
    publish_if_needed(s, stream);
    for (int64_t n = 0; n < nsteps; ++n) {
      enqueue_steps(s, 1, stream);
      launch_probe_energy(s, dev(s, s.L.Y), pd, nprobe, s.dt, Jd, stream);
    }
    hip_check(hipStreamSynchronize(st), "sync");
    s.nstep += nsteps;
    hip_check(hipMemcpy(J, Jd, 8, hipMemcpyDeviceToHost), "J");
  });
}

mdg_status mdg_probe_energy_noalloc(mdg_solver* h, int64_t nsteps, int32_t nprobe, const int64_t* probes, double* J,
                                    void* stream) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (nsteps < 0) throw Error(MDG_E_ARG, "probe energy: nsteps >= 0");
    if (nprobe < 1 || !probes || !J) throw Error(MDG_E_ARG, "probe energy: probes and J required");
    if (nprobe > MDG_NOALLOC_MAX_PROBES)
      throw Error(MDG_E_ARG, "probe_energy_noalloc: nprobe > MDG_NOALLOC_MAX_PROBES (" +
                                 std::to_string(MDG_NOALLOC_MAX_PROBES) + ")");
    int64_t pin[MDG_NOALLOC_MAX_PROBES];
    for (int i = 0; i < nprobe; ++i) {
      if (probes[i] < 0 || probes[i] >= s.nt) throw Error(MDG_E_ARG, "probe energy: element out of range");
      pin[i] = s.iperm[probes[i]];
    }
    unsigned char* base = scratch_ptr();
    double* Jd = reinterpret_cast<double*>(base);
    int64_t* pd = reinterpret_cast<int64_t*>(base + 256);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hip_check(hipMemcpyAsync(pd, pin, size_t(nprobe) * 8, hipMemcpyHostToDevice, st), "probes");
    hipLaunchKernelGGL(zero_one, dim3(1), dim3(64), 0, st, Jd);
    hip_check(hipGetLastError(), "zero_one launch");
    publish_if_needed(s, stream);
    for (int64_t n = 0; n < nsteps; ++n) {
      enqueue_steps(s, 1, stream);
      launch_probe_energy(s, dev(s, s.L.Y), pd, nprobe, s.dt, Jd, stream);
    }
    hip_check(hipStreamSynchronize(st), "sync");
    s.nstep += nsteps;
    hip_check(hipMemcpy(J, Jd, 8, hipMemcpyDeviceToHost), "J");
  });
}

mdg_status mdg_adjoint_probe_energy(mdg_solver* h, int64_t nsteps, int32_t every, int32_t nprobe,
                                     const int64_t* probes, double* J, double* grad_eps, void* stream) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (nsteps < 1 || every < 1) throw Error(MDG_E_ARG, "adjoint: nsteps >= 1 and checkpoint interval >= 1");
    if (nprobe < 1 || !probes || !J || !grad_eps) throw Error(MDG_E_ARG, "adjoint: probes, J and grad_eps required");
    if (s.opt.integrator != MDG_RK4) throw Error(MDG_E_UNSUPPORTED, "adjoint: RK4 steps only");
    std::vector<int64_t> pin(nprobe);
    for (int i = 0; i < nprobe; ++i) {
      if (probes[i] < 0 || probes[i] >= s.nt) throw Error(MDG_E_ARG, "adjoint: probe element out of range");
      pin[i] = s.iperm[probes[i]];
    }
    // a state vector: fields (blocked layout), with PML elements the
    // auxiliaries of the PML elements, with SIP the surface unknown
    const bool pml = s.Kp > 0, upw = s.opt.flux == MDG_UPWIND, sip = s.sip();
    const size_t SB = size_t(state_rows(s)) * s.Kpad * s.real_size();
    const size_t SA = pml ? size_t(state_rows(s)) * s.Kppad * s.real_size() : 0;
    const size_t SS = sip ? size_t(8) * s.NF * s.Kpad * s.real_size() : 0;
    struct SV {
      void* u = nullptr;
      void* q = nullptr;
      void* s = nullptr;
    };
    DevBufs B;
    hipStream_t st = static_cast<hipStream_t>(stream);
    auto alloc = [&]() {
      SV v;
      v.u = B.get(SB);
      if (pml) v.q = B.get(SA);
      if (sip) v.s = B.get(SS);
      return v;
    };
    auto copy = [&](SV d, SV x) {
      hip_check(hipMemcpyAsync(d.u, x.u, SB, hipMemcpyDeviceToDevice, st), "adjoint copy");
      if (pml) hip_check(hipMemcpyAsync(d.q, x.q, SA, hipMemcpyDeviceToDevice, st), "adjoint copy");
      if (sip) hip_check(hipMemcpyAsync(d.s, x.s, SS, hipMemcpyDeviceToDevice, st), "adjoint copy");
    };
    const int64_t k = std::min<int64_t>(every, nsteps);
    const int64_t nseg = (nsteps + k - 1) / k;
    // checkpoints u^{j k}; per step n of the segment being reversed its state
    // x_n (seg, one more for the segment's end) and its stage derivatives
    // K_1..K_4, stored by the recomputation (device memory: 5 k + 6 + nseg
    // state vectors); the adjoint stepping arrays (nu is its base state)
    std::vector<SV> ck(nseg), seg(k + 1);
    std::vector<std::array<SV, 4>> Ks(k);
    for (auto& q : ck) q = alloc();
    for (auto& q : seg) q = alloc();
    for (auto& st4 : Ks)
      for (auto& q : st4) q = alloc();
    const SV nu = alloc(), aUa = alloc(), aUb = alloc(), aAcc = alloc(), uend = alloc();
    SV state;
    state.u = dev(s, s.L.Y);
    state.q = pml ? dev(s, s.L.aY) : nullptr;
    state.s = sip ? dev(s, s.L.sY) : nullptr;
    double* g = static_cast<double*>(B.get(size_t(s.K) * 8));
    double* Jd = static_cast<double*>(B.get(8));
    int64_t* pd = static_cast<int64_t*>(B.get(size_t(nprobe) * 8));
    hip_check(hipMemcpyAsync(pd, pin.data(), pin.size() * 8, hipMemcpyHostToDevice, st), "probes");
    hip_check(hipMemsetAsync(g, 0, size_t(s.K) * 8, st), "grad");
    hip_check(hipMemsetAsync(Jd, 0, 8, st), "J");
    const double dt = s.dt;
    const int64_t nbase = s.nstep;
    // the time of every step on the device, (t0, n): stage times t0 + (n + c) dt
    double* clk = static_cast<double*>(B.get(size_t(16) * nsteps));
    {
      std::vector<double> c(size_t(2) * nsteps);
      for (int64_t n = 0; n < nsteps; ++n) {
        c[2 * n] = s.t0;
        c[2 * n + 1] = double(nbase + n);
      }
      hip_check(hipMemcpyAsync(clk, c.data(), c.size() * 8, hipMemcpyHostToDevice, st), "clocks");
      hip_check(hipStreamSynchronize(st), "sync");
    }
    // forward: J and checkpoints u^{j k}
    publish_if_needed(s, stream);
    for (int64_t n = 0; n < nsteps; ++n) {
      if (n % k == 0) copy(ck[n / k], state);
      enqueue_steps(s, 1, stream);
      launch_probe_energy(s, state.u, pd, nprobe, dt, Jd, stream);
    }
    copy(uend, state);
    // reverse sweep in nu = M^-1 lambda (M: the mass, auxiliaries weighted
    // like their field). With a_i the adjoint stage vectors of the RK4 step
    // and m_i = L* a_i, L* = M^-1 L^T M, the scaled vectors a_i / (b_i dt) are
    // the stage inputs of one classic RK4 step of L* (with its stages in
    // reverse order: a_4 / (b_4 dt) = nu, a_3 / (b_3 dt) = nu + dt/2 m_4 / (b_4 dt),
    // ...), and the update nu + sum_i m_i is that step's result: the adjoint of
    // a step is one fused RK4 step of the adjoint operator, which the stage
    // kernel evaluates directly (skew part negated, PML couplings transposed)
    hip_check(hipMemsetAsync(nu.u, 0, SB, st), "nu");
    if (pml) hip_check(hipMemsetAsync(nu.q, 0, SA, st), "nu");
    if (sip) hip_check(hipMemsetAsync(nu.s, 0, SS, st), "nu");
    launch_probe_add(s, nu.u, uend.u, pd, nprobe, dt, stream);
    const DevLayout& L = s.L;
    const RKBufs ab{nu.u, aUa.u, aUb.u, aAcc.u, nu.q, aUa.q, aUb.q, aAcc.q, nu.s, aUa.s, aUb.s, aAcc.s};
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
      const int64_t n0 = sgi * k, n1 = std::min(nsteps, n0 + k);
      // recompute the segment from its checkpoint by the stepping launches,
      // each step from seg[j] into seg[j + 1], its stage derivatives into Ks[j]
      copy(seg[0], ck[sgi]);
      launch_publish(s, seg[0].u, dev(s, L.H0), stream);
      for (int64_t j = 0; j < n1 - n0; ++j) {
        RKBufs rb = solver_bufs(s);
        rb.Y = seg[j].u;
        rb.aY = seg[j].q;
        rb.sY = seg[j].s;
        rb.Yout = seg[j + 1].u;
        rb.aYout = seg[j + 1].q;
        rb.sYout = seg[j + 1].s;
        for (int i = 0; i < 4; ++i) {
          rb.K[i] = Ks[j][i].u;
          rb.aK[i] = Ks[j][i].q;
          rb.sK[i] = Ks[j][i].s;
        }
        enqueue_rk4_step(s, rb, clk + 2 * (n0 + j), true, false, nullptr, stream,
                         [](int, const void*, const void*, const void*) {});
      }
      // the halo traces of nu (the recomputation used the halo buffers); each
      // adjoint step leaves those of its result in H0, and after the probe
      // term only the probe elements' traces change
      launch_publish(s, nu.u, dev(s, L.H0), stream);
      for (int64_t n = n1 - 1; n >= n0; --n) {
        const SV x = seg[n - n0];
        const std::array<SV, 4>& K = Ks[n - n0];
        // the adjoint step; before its stage i (input a_{4-i} / (b_{4-i} dt))
        // the gradient takes g -= (a, K_curl)_M0 over the E rows with the
        // forward stage f = 4-i (only the curl part of K scales with 1/eps;
        // PML elements add the damping part back) and, with the upwind flux,
        // g += (a, dA/deps X) for the face impedances, X_f = x + c_f dt K_{f-1}
        // the forward stage input
        enqueue_rk4_step(s, ab, clk + 2 * n, false, true, nullptr, stream,
                         [&](int i, const void* in, const void*, const void*) {
                           const int f = 3 - i;  // forward stage
                           const double sc = RK_B[f] * dt, cf = RK_C[f] * dt;
                           const SV kp = f ? K[f - 1] : SV{};
                           launch_grad_stage(s, g, in, K[f].u, x.u, kp.u, x.q, kp.q, cf, sc, stream);
                           if (upw) launch_grad_upw(s, g, in, x.u, kp.u, cf, sc, stream);
                         });
        if (n >= 1) {
          launch_probe_add(s, nu.u, x.u, pd, nprobe, dt, stream);
          launch_publish(s, nu.u, dev(s, L.H0), stream, pd, nprobe);
        }
      }
    }
    // the solver state is the forward end state
    copy(state, uend);
    hip_check(hipStreamSynchronize(st), "sync");
    s.nstep = nbase + nsteps;
    set_clock(s, s.L.clock, s.t0, double(s.nstep));
    s.halo_valid = false;
    std::vector<double> gh(s.K);
    hip_check(hipMemcpy(gh.data(), g, size_t(s.K) * 8, hipMemcpyDeviceToHost), "grad");
    hip_check(hipMemcpy(J, Jd, 8, hipMemcpyDeviceToHost), "J");
    for (int64_t u = 0; u < s.nt; ++u) grad_eps[u] = gh[s.iperm[u]];
  });
}

mdg_status mdg_energy(mdg_solver* h, double* W) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (!W) throw Error(MDG_E_ARG, "NULL W");
    hip_check(hipDeviceSynchronize(), "synchronize");
    launch_energy(s, dev(s, s.L.Y), nullptr);
    hip_check(hipMemcpy(W, dev(s, s.L.eout), sizeof(double), hipMemcpyDeviceToHost), "energy copy");
    if (!std::isfinite(*W)) throw Error(MDG_E_UNSTABLE, "energy is not finite");
  });
}

mdg_status mdg_energy_instances(mdg_solver* h, double* W) {
  return guarded(h, [&](Solver& s) {
    need_bound(s);
    if (!W) throw Error(MDG_E_ARG, "NULL W");
    hip_check(hipDeviceSynchronize(), "synchronize");
    launch_energy(s, dev(s, s.L.Y), nullptr);
    std::vector<double> e(s.K);
    hip_check(hipMemcpy(e.data(), dev(s, s.L.eelem), s.K * sizeof(double), hipMemcpyDeviceToHost), "energy copy");
    const int ni = (int)s.inst_first.size() - 1;
    for (int i = 0; i < ni; ++i) {
      double w = 0.0;
      for (int64_t k = s.inst_first[i]; k < s.inst_first[i + 1]; ++k) w += e[s.iperm[k]];
      if (!std::isfinite(w)) throw Error(MDG_E_UNSTABLE, "energy is not finite");
      W[i] = w;
    }
  });
}

mdg_status mdg_query(mdg_solver* h, mdg_info* info) {
  return guarded(h, [&](Solver& s) {
    if (!info) throw Error(MDG_E_ARG, "NULL info");
    std::memset(info, 0, sizeof(*info));
    info->order = s.P;
    info->nmodes = s.N;
    info->order_h = s.P - (s.NH < s.N ? 1 : 0);
    info->nmodes_h = s.NH;
    info->nfacemodes = s.NF;
    info->precision = s.opt.precision;
    info->flux = s.opt.flux;
    if (s.nt == 0) return;
    ensure_final(s);
    info->tile_size = s.tile;
    info->n_elements = s.nt;
    info->n_faces_interior = s.n_int;
    info->n_faces_boundary = s.n_bnd;
    info->n_pml = s.Kp;
    info->n_tiles = s.ntiles;
    info->n_halo = s.nhalo;
    info->dt = s.bound ? s.dt : (s.opt.dt > 0 ? s.opt.dt : cfl_dt(s));
    info->time = s.time();
    info->n_instances = (int64_t)s.inst_first.size() - 1;
    info->n_dipoles = (int64_t)s.dips.size();
    info->bytes_per_stage = bytes_per_stage(s);
    info->flops_per_stage = flops_per_stage(s);
    info->workspace_bytes = (int64_t)s.L.total;
  });
}

}  // extern "C"

// stage_launch.hip -- host dispatch of the stage, energy, publication and
// upwind-gradient launches to the (precision, order) instances, and the two
// small precision-independent kernels (dipole amplitudes, energy total).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "stage_args.hpp"

namespace mdg {

static void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// dipole amplitudes at the times t = t0 + (n + c_j) dt of the device clock,
// j < ns, into amp[j][d]: the Gaussian-modulated sinusoid
// g(t) = sin(2 pi f0 (t - tc)) exp(-(t - tc)^2 / (2 s^2)), s = 1/(2 pi bw), in FP64
struct StageTimes {
  double c[4];
};
__global__ __launch_bounds__(256) void src_amp_kernel(const double* __restrict__ clock, StageTimes cs, int ns, double dt,
                                                      const double* __restrict__ wave, int nd,
                                                      double* __restrict__ amp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ns * nd) return;
  const int j = i / nd, d = i - j * nd;
  const double t = clock[0] + (clock[1] + cs.c[j]) * dt;
  const double pi = 3.14159265358979323846;
  const double tau = t - wave[3 * d + 2], sg = 1.0 / (2.0 * pi * wave[3 * d + 1]);
  amp[i] = sin(2.0 * pi * wave[3 * d] * tau) * exp(-tau * tau / (2.0 * sg * sg));
}

__global__ __launch_bounds__(256) void energy_final(const double* __restrict__ part, int64_t n,
                                                    double* __restrict__ out) {
  __shared__ double red[4];
  double w = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) w += part[i];
  for (int o = 32; o > 0; o >>= 1) w += __shfl_down(w, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

template <typename R>
static void launch_r(int P, const DevArgs& a, bool upw, bool sip, bool pml, int tile, size_t lds, bool mfma,
                     bool ps, bool mix, hipStream_t st) {
  switch (P) {
    case 1: launch_p<R, 1>(a, upw, sip, pml, tile, lds, mfma, ps, mix, st); break;
    case 2: launch_p<R, 2>(a, upw, sip, pml, tile, lds, mfma, ps, mix, st); break;
    case 3: launch_p<R, 3>(a, upw, sip, pml, tile, lds, mfma, ps, mix, st); break;
    case 4: launch_p<R, 4>(a, upw, sip, pml, tile, lds, mfma, ps, mix, st); break;
    default: throw Error(MDG_E_UNSUPPORTED, "order not compiled");
  }
}

void launch_stage(const Solver& s, const StageParams& sp, void* stream) {
  char* base = static_cast<char*>(s.ws);
  DevArgs a{};
  // the first RK4 stage reads its base state as its input (the FP64 kernel
  // takes y from the staged input there)
  if (sp.stage == 0 && sp.Uin != sp.Y) throw Error(MDG_E_STATE, "RK4 stage 0 takes the base state as its input");
  // the final RK4 stage writes the new state through Uout: into Yout, or in place
  const bool fin = sp.stage == 3;
  a.Y = sp.Y;
  a.Uin = sp.Uin;
  a.Uout = fin ? (sp.Yout ? sp.Yout : sp.Y) : sp.Uout;
  a.Kout = sp.Kout;
  a.ACC = sp.ACC;
  a.aY = sp.aY;
  a.aYw = sp.aY;
  a.aUin = sp.aUin;
  a.aUout = fin ? (sp.aYout ? sp.aYout : sp.aY) : sp.aUout;
  a.aKout = sp.aKout;
  a.aACC = sp.aACC;
  a.sY = sp.sY;
  a.sUin = sp.sUin;
  a.sUout = fin ? (sp.sYout ? sp.sYout : sp.sY) : sp.sUout;
  a.sKout = sp.sKout;
  a.sACC = sp.sACC;
  a.geo = base + s.L.geo;
  a.nbr = reinterpret_cast<const int32_t*>(base + s.L.nbr);
  a.pub = reinterpret_cast<const int32_t*>(base + s.L.pub);
  a.halo_tile = reinterpret_cast<const int32_t*>(base + s.L.halo_tile);
  a.hin = sp.hin;
  a.hout = sp.hout;
  a.publish = sp.publish && sp.hout != nullptr;
  a.pml = base + s.L.pml;
  a.src = base + s.L.src;
  a.srcid = reinterpret_cast<const int32_t*>(base + s.L.srcid);
  a.srcnext = reinterpret_cast<const int32_t*>(base + s.L.srcnext);
  a.srcamp = reinterpret_cast<const double*>(base + s.L.srcamp);
  a.has_src = (sp.sources && !s.dips.empty()) ? 1 : 0;
  const size_t rs = s.real_size();
  a.nblk = (uint32_t)(s.Kpad / 64);
  a.pnblk = (uint32_t)(s.Kppad / 64);
  a.hbuf_bytes = (uint32_t)(size_t(s.hbuf_reals) * rs);
  a.sip = s.sip() ? 1 : 0;
  if (s.sip() && !(sp.sY && sp.sUin && (sp.stage >= 3 || sp.sUout) && (sp.stage < 0 || sp.stage > 3 || sp.sACC)))
    throw Error(MDG_E_STATE, "SIP launch without its surface buffers");
  a.pml_base = s.K0;
  a.nh = s.NH;
  a.nfh = s.NFH;
  a.hreg = (int32_t)s.hreg;
  a.adj = sp.adj ? 1 : 0;
  a.stage = sp.stage;
  a.bcoef = sp.bcoef;
  a.cdt = sp.cdt;
  a.dt = sp.dt;
  const bool fp32 = s.opt.precision == MDG_FP32;
  const bool upw = s.opt.flux == MDG_UPWIND;
  const LdsLayout ll = stage_lds_layout(s, sp.stage >= 4 && s.tile % 64 == 0);
  const size_t lds = ll.bytes;
  a.stg_base = ll.stg_base;
  a.halo_base = ll.halo_base;
  a.out_base = ll.out_base;
  a.tile = s.tile;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (a.has_src) {
    // the amplitudes of all four stages of an RK4 step are evaluated before
    // its first stage (the clock advances in its last), those of any other
    // launch before it
    const int nd = (int)s.dips.size();
    const bool rk = sp.stage >= 0 && sp.stage <= 3;
    double* amp = reinterpret_cast<double*>(base + s.L.srcamp);
    if (!rk || sp.stage == 0) {
      const int ns = rk ? 4 : 1;
      const StageTimes cs = rk ? StageTimes{{0.0, 0.5, 0.5, 1.0}} : StageTimes{{sp.cstage, 0.0, 0.0, 0.0}};
      hipLaunchKernelGGL(src_amp_kernel, dim3((ns * nd + 255) / 256), dim3(256), 0, st, sp.clock, cs, ns, sp.dt,
                         reinterpret_cast<const double*>(base + s.L.srcwave), nd, amp);
      hip_check(hipGetLastError(), "src_amp_kernel launch");
    }
    a.srcamp = amp + (rk ? sp.stage : 0) * nd;
  }
  // non-PML tiles, then PML tiles; the last launch carries the clock tick
  const int last = s.ntiles > s.ntiles0 ? 1 : 0;
  for (int part = 0; part < 2; ++part) {
    a.tick = part == last ? sp.tick : nullptr;
    a.tile_begin = part == 0 ? 0 : (int32_t)s.ntiles0;
    a.elem_begin = part == 0 ? 0 : (int32_t)s.K0;
    a.elem_end = part == 0 ? (int32_t)s.K0 : (int32_t)s.K;
    a.ntiles = part == 0 ? (int32_t)s.ntiles0 : (int32_t)(s.ntiles - s.ntiles0);
    if (a.ntiles == 0) continue;
    const bool ps = s.opt.launch == MDG_LAUNCH_PERSISTENT;
    const bool mix = s.NH < s.N;
    if (fp32) launch_r<float>(s.P, a, upw, s.sip(), part == 1, s.tile, lds, s.opt.mfma != 0, ps, mix, st);
    else launch_r<double>(s.P, a, upw, s.sip(), part == 1, s.tile, lds, s.opt.mfma != 0, ps, mix, st);
  }
}

template <typename R>
static void launch_energy_r(const Solver& s, const void* Y, hipStream_t st) {
  char* base = static_cast<char*>(s.ws);
  double* part = reinterpret_cast<double*>(base + s.L.epart);
  double* ee = reinterpret_cast<double*>(base + s.L.eelem);
  const void* geo = base + s.L.geo;
  switch (s.P) {
    case 1: launch_energy_rp<R, 1>(Y, geo, s.K, part, ee, s.NH, st); break;
    case 2: launch_energy_rp<R, 2>(Y, geo, s.K, part, ee, s.NH, st); break;
    case 3: launch_energy_rp<R, 3>(Y, geo, s.K, part, ee, s.NH, st); break;
    case 4: launch_energy_rp<R, 4>(Y, geo, s.K, part, ee, s.NH, st); break;
    default: throw Error(MDG_E_UNSUPPORTED, "order not compiled");
  }
  const int64_t nblk = (s.K + 255) / 256;
  hipLaunchKernelGGL(energy_final, dim3(1), dim3(256), 0, st, part, nblk, reinterpret_cast<double*>(base + s.L.eout));
  hip_check(hipGetLastError(), "energy_final launch");
}

void launch_energy(const Solver& s, const void* Y, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s.opt.precision == MDG_FP32) launch_energy_r<float>(s, Y, st);
  else launch_energy_r<double>(s, Y, st);
}

// mon = [last energy, flag (0 ok, 1 growth, 2 not finite), first energy, latest energy]
__global__ void monitor_kernel(const double* __restrict__ W, double* __restrict__ mon, int init, int growth,
                               double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double w = W[0];
  if (init) {
    mon[1] = 0.0;
    mon[2] = w;
  } else if (growth && w > mon[0] * (1.0 + tol) && mon[1] == 0.0) {
    mon[1] = 1.0;
  }
  if (!(w - w == 0.0)) mon[1] = 2.0;  // NaN or infinite
  mon[0] = w;
  mon[3] = w;
}

void launch_monitor(const Solver& s, bool init, bool growth, double tol, void* stream) {
  char* base = static_cast<char*>(s.ws);
  hipLaunchKernelGGL(monitor_kernel, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const double*>(base + s.L.eout), reinterpret_cast<double*>(base + s.L.mon),
                     init ? 1 : 0, growth ? 1 : 0, tol);
  hip_check(hipGetLastError(), "monitor_kernel launch");
}

template <typename R>
static void launch_publish_r(const Solver& s, const void* U, void* H, const int64_t* list, int nlist,
                             hipStream_t st) {
  char* base = static_cast<char*>(s.ws);
  const size_t rs = s.real_size();
  const uint32_t nblk = (uint32_t)(s.Kpad / 64);
  const uint32_t hb = (uint32_t)(size_t(s.hbuf_reals) * rs);
  const int32_t* pub = reinterpret_cast<const int32_t*>(base + s.L.pub);
  const int K = (int)s.K, hreg = (int)s.hreg;
  switch (s.P) {
    case 1: launch_publish_rp<R, 1>(U, nblk, s.NH, pub, H, hb, K, hreg, list, nlist, st); break;
    case 2: launch_publish_rp<R, 2>(U, nblk, s.NH, pub, H, hb, K, hreg, list, nlist, st); break;
    case 3: launch_publish_rp<R, 3>(U, nblk, s.NH, pub, H, hb, K, hreg, list, nlist, st); break;
    case 4: launch_publish_rp<R, 4>(U, nblk, s.NH, pub, H, hb, K, hreg, list, nlist, st); break;
    default: throw Error(MDG_E_UNSUPPORTED, "order not compiled");
  }
}

void launch_publish(const Solver& s, const void* U, void* H, void* stream, const int64_t* list, int nlist) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (s.nhalo == 0) return;
  if (s.opt.precision == MDG_FP32) launch_publish_r<float>(s, U, H, list, nlist, st);
  else launch_publish_r<double>(s, U, H, list, nlist, st);
}

void launch_grad_upw(const Solver& s, double* g, const void* a, const void* x, const void* dx, double c,
                     double scale, void* stream) {
  char* base = static_cast<char*>(s.ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int32_t* nb = reinterpret_cast<const int32_t*>(base + s.L.nbrg);
  const void* geo = base + s.L.geo;
#define MDG_UPW(R, P) launch_grad_upw_rp<R, P>(g, a, x, dx, c, geo, nb, s.K, scale, s.NH, st)
  const bool fp32 = s.opt.precision == MDG_FP32;
  switch (s.P) {
    case 1: if (fp32) MDG_UPW(float, 1); else MDG_UPW(double, 1); break;
    case 2: if (fp32) MDG_UPW(float, 2); else MDG_UPW(double, 2); break;
    case 3: if (fp32) MDG_UPW(float, 3); else MDG_UPW(double, 3); break;
    case 4: if (fp32) MDG_UPW(float, 4); else MDG_UPW(double, 4); break;
    default: throw Error(MDG_E_UNSUPPORTED, "order not compiled");
  }
#undef MDG_UPW
}

}  // namespace mdg

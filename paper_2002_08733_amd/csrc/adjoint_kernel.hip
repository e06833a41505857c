// adjoint_kernel.hip -- device kernels of the discrete adjoint of the RK4
// trajectory (probe-energy objective, gradient w.r.t. per-element eps): the
// probe energy and its derivative, and the per-element gradient
// accumulation. The forward stage values and the adjoint steps themselves are
// stage-kernel launches (stage_kernel.hip).
//
// All state vectors use the blocked layout of the stage kernel:
// [K/64][field E,H][3N rows][64], row = component*N + mode. The covariant
// mass of element T is M_T = eps_T M0_T (E) / mu_T M0_T (H) per mode with
// M0_T = |det A| A^-1 A^-T = (G0^-1)^-1, G0^-1 the geometry record.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "solver.hpp"

namespace mdg {

// M0 of element k from its geometry record
template <typename R>
__device__ __forceinline__ void mass0(const R* __restrict__ geo, int64_t k, double (&m)[6]) {
  const R* gk = geo + (k >> 6) * NGEO * 64 + (k & 63);
  const double a = gk[G_XX * 64], b = gk[G_XY * 64], c = gk[G_XZ * 64];
  const double d = gk[G_YY * 64], e = gk[G_YZ * 64], f = gk[G_ZZ * 64];
  const double det = a * (d * f - e * e) - b * (b * f - e * c) + c * (b * e - d * c);
  const double id = 1.0 / det;
  m[0] = (d * f - e * e) * id;  // xx
  m[1] = (c * e - b * f) * id;  // xy
  m[2] = (b * e - c * d) * id;  // xz
  m[3] = (a * f - c * c) * id;  // yy
  m[4] = (b * c - a * e) * id;  // yz
  m[5] = (a * d - b * b) * id;  // zz
}

// (u, v)_{M0, E, T} = sum_l u_l^T M0_T v_l over the E rows of element k
template <typename R, int N>
__device__ __forceinline__ double e_dot(const R* __restrict__ u, const R* __restrict__ v, const double (&m)[6],
                                        int64_t k, int64_t rb) {
  const R* uk = u + (k >> 6) * rb * 64 + (k & 63);
  const R* vk = v + (k >> 6) * rb * 64 + (k & 63);
  double s = 0.0;
  for (int l = 0; l < N; ++l) {
    const double ux = uk[(0 * N + l) * 64], uy = uk[(1 * N + l) * 64], uz = uk[(2 * N + l) * 64];
    const double vx = vk[(0 * N + l) * 64], vy = vk[(1 * N + l) * 64], vz = vk[(2 * N + l) * 64];
    s += ux * (m[0] * vx + m[1] * vy + m[2] * vz) + uy * (m[1] * vx + m[3] * vy + m[4] * vz) +
         uz * (m[2] * vx + m[4] * vy + m[5] * vz);
  }
  return s;
}

// J += dt sum_{probes} (e, e)_{M0}: one block, fixed summation order
template <typename R, int N>
__global__ __launch_bounds__(256) void probe_energy_kernel(const R* __restrict__ u, const R* __restrict__ geo,
                                                           const int64_t* __restrict__ probes, int np, double dt,
                                                           double* __restrict__ J, int64_t rb) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    double m[6];
    mass0(geo, probes[i], m);
    s += e_dot<R, N>(u, u, m, probes[i], rb);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] += dt * red[0];
}

// nu_E += (2 dt / eps_T) u_E on the probe elements (the derivative of the
// probe energy, mapped by M^-1)
template <typename R, int N>
__global__ __launch_bounds__(256) void probe_add_kernel(R* __restrict__ nu, const R* __restrict__ u,
                                                        const R* __restrict__ geo, const int64_t* __restrict__ probes,
                                                        int np, double dt, int64_t rb) {
  const int i = blockIdx.x;
  if (i >= np) return;
  const int64_t k = probes[i];
  const R* gk = geo + (k >> 6) * NGEO * 64 + (k & 63);
  const double f = 2.0 * dt * (double)gk[G_IEPS * 64];
  const int64_t base = (k >> 6) * rb * 64 + (k & 63);
  for (int r = threadIdx.x; r < 3 * N; r += 256) nu[base + r * 64] = (R)((double)nu[base + r * 64] + f * (double)u[base + r * 64]);
}

// One forward stage of the reverse sweep, for every element T:
//   g_T -= scale (a, K)_{M0, E, T}
// and on the PML elements (k >= K0) the damping part of the stage derivative,
// which does not scale with 1/eps, added back (with it g_T gets
// -(a, K_curl)_M0 where K_curl = K + A^T (eta c + q) is the part that does):
//   g_T -= scale (a, A^T (eta c + q))_{M0, E, T},  c = A^-T x_E,
// q the scaled Cartesian auxiliary, (x, xa) + cs (dx, dxa) the forward stage
// input (dx, dxa null: cs = 0). Four lanes per element, lane j taking the
// modes l = j, j + 4, ...; the partial sums meet by shuffles in a fixed order.
template <typename R, int N>
__global__ __launch_bounds__(256) void grad_stage_kernel(double* __restrict__ g, const R* __restrict__ a,
                                                         const R* __restrict__ K, const R* __restrict__ x,
                                                         const R* __restrict__ dx, const R* __restrict__ xa,
                                                         const R* __restrict__ dxa, double cs,
                                                         const R* __restrict__ geo, const R* __restrict__ pml,
                                                         int64_t nk, int64_t K0, double scale, int64_t rb) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t k = t >> 2;
  const int j = (int)(t & 3);
  double s = 0.0;  // lanes past the last element add nothing but join the shuffles
  if (k < nk) {
    double m[6];
    mass0(geo, k, m);
    const int64_t ok = (k >> 6) * rb * 64 + (k & 63);
    const R* ak = a + ok;
    const R* kk = K + ok;
    auto mdot = [&](const double (&v)[3], const double (&z)[3]) {
      return v[0] * (m[0] * z[0] + m[1] * z[1] + m[2] * z[2]) + v[1] * (m[1] * z[0] + m[3] * z[1] + m[4] * z[2]) +
             v[2] * (m[2] * z[0] + m[4] * z[1] + m[5] * z[2]);
    };
    for (int l = j; l < N; l += 4) {
      double v[3], z[3];
      for (int c = 0; c < 3; ++c) {
        v[c] = ak[(c * N + l) * 64];
        z[c] = kk[(c * N + l) * 64];
      }
      s += mdot(v, z);
    }
    if (k >= K0) {
      const int64_t pk = k - K0, oq = (pk >> 6) * rb * 64 + (pk & 63);
      const R* pr = pml + (pk >> 6) * NPML * 64 + (pk & 63);
      double AT[9], AiT[9];
      for (int i = 0; i < 9; ++i) {
        AT[i] = pr[(PM_AT + i) * 64];
        AiT[i] = pr[(PM_AIT + i) * 64];
      }
      const double wx = pr[(PM_OM + 0) * 64], wy = pr[(PM_OM + 1) * 64], wz = pr[(PM_OM + 2) * 64];
      const double eta[3] = {wy + wz - wx, wz + wx - wy, wx + wy - wz};
      auto xv = [&](int r) { return (double)x[ok + r * 64] + (dx ? cs * (double)dx[ok + r * 64] : 0.0); };
      auto qv = [&](int r) { return (double)xa[oq + r * 64] + (dxa ? cs * (double)dxa[oq + r * 64] : 0.0); };
      for (int l = j; l < N; l += 4) {
        double u[3], y[3], z[3], v[3];
        for (int c = 0; c < 3; ++c) u[c] = xv(c * N + l);
        for (int i = 0; i < 3; ++i)
          y[i] = eta[i] * (AiT[3 * i] * u[0] + AiT[3 * i + 1] * u[1] + AiT[3 * i + 2] * u[2]) + qv(i * N + l);
        for (int c = 0; c < 3; ++c) z[c] = AT[3 * c] * y[0] + AT[3 * c + 1] * y[1] + AT[3 * c + 2] * y[2];
        for (int c = 0; c < 3; ++c) v[c] = ak[(c * N + l) * 64];
        s += mdot(v, z);
      }
    }
  }
  s += __shfl_xor(s, 1, 64);
  s += __shfl_xor(s, 2, 64);
  if (j == 0 && k < nk) g[k] -= scale * s;
}

// ---------------------------------------------------------------- launch
static void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define MDG_BY_ORDER(R, KERNEL, ...)                                                  \
  switch (s.P) {                                                                      \
    case 1: hipLaunchKernelGGL((KERNEL<R, 4>), __VA_ARGS__); break;                  \
    case 2: hipLaunchKernelGGL((KERNEL<R, 10>), __VA_ARGS__); break;                 \
    case 3: hipLaunchKernelGGL((KERNEL<R, 20>), __VA_ARGS__); break;                 \
    case 4: hipLaunchKernelGGL((KERNEL<R, 35>), __VA_ARGS__); break;                 \
    default: throw Error(MDG_E_UNSUPPORTED, "order not compiled");                    \
  }

void launch_probe_energy(const Solver& s, const void* u, const int64_t* probes, int np, double dt, double* J,
                         void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void* geo = static_cast<char*>(s.ws) + s.L.geo;
  const int64_t rb = state_rows(s);
  if (s.opt.precision == MDG_FP32) {
    MDG_BY_ORDER(float, probe_energy_kernel, dim3(1), dim3(256), 0, st, (const float*)u, (const float*)geo, probes,
                 np, dt, J, rb)
  } else {
    MDG_BY_ORDER(double, probe_energy_kernel, dim3(1), dim3(256), 0, st, (const double*)u, (const double*)geo,
                 probes, np, dt, J, rb)
  }
  check(hipGetLastError(), "probe_energy_kernel launch");
}

void launch_probe_add(const Solver& s, void* nu, const void* u, const int64_t* probes, int np, double dt,
                      void* stream) {
  if (np == 0) return;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void* geo = static_cast<char*>(s.ws) + s.L.geo;
  const int64_t rb = state_rows(s);
  if (s.opt.precision == MDG_FP32) {
    MDG_BY_ORDER(float, probe_add_kernel, dim3(np), dim3(256), 0, st, (float*)nu, (const float*)u, (const float*)geo,
                 probes, np, dt, rb)
  } else {
    MDG_BY_ORDER(double, probe_add_kernel, dim3(np), dim3(256), 0, st, (double*)nu, (const double*)u,
                 (const double*)geo, probes, np, dt, rb)
  }
  check(hipGetLastError(), "probe_add_kernel launch");
}

void launch_grad_stage(const Solver& s, double* g, const void* a, const void* K, const void* x, const void* dx,
                       const void* xa, const void* dxa, double c, double scale, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void* geo = static_cast<char*>(s.ws) + s.L.geo;
  const void* pml = static_cast<char*>(s.ws) + s.L.pml;
  const dim3 grid((unsigned)((4 * s.K + 255) / 256));
  const int64_t rb = state_rows(s);
  const int64_t K0 = s.Kp > 0 ? s.K0 : s.K;  // no damped elements: no damping part
  if (s.opt.precision == MDG_FP32) {
    MDG_BY_ORDER(float, grad_stage_kernel, grid, dim3(256), 0, st, g, (const float*)a, (const float*)K,
                 (const float*)x, (const float*)dx, (const float*)xa, (const float*)dxa, c, (const float*)geo,
                 (const float*)pml, s.K, K0, scale, rb)
  } else {
    MDG_BY_ORDER(double, grad_stage_kernel, grid, dim3(256), 0, st, g, (const double*)a, (const double*)K,
                 (const double*)x, (const double*)dx, (const double*)xa, (const double*)dxa, c,
                 (const double*)geo, (const double*)pml, s.K, K0, scale, rb)
  }
  check(hipGetLastError(), "grad_stage_kernel launch");
}
#undef MDG_BY_ORDER

}  // namespace mdg

// stage_kernel.hpp -- fused RK4 stage of the matrix-free DG Maxwell operator
// for gfx950 (CDNA4), plus the FP64 energy reduction.
//
// One launch applies the semi-discrete operator [KS Sec. III-IV] to the stage
// input of every element and performs that stage's RK4 update in the epilogue.
//
// Work decomposition
//   * Elements are ordered by recursive coordinate bisection of their
//     centroids (PML elements last) and cut into tiles of TILE consecutive
//     elements (64, or 32 where the LDS of the trace exchange would be too
//     large: FP64 from order 2, FP32 order 4); one workgroup per tile. Eight lanes
//     per element: two roles x four parts. Role 0 produces the E update and
//     reads H as its volume input, role 1 the H update from E:
//        r_E = +s W(h) - Lift(h~) + Pen_Z([e]),   r_H = -s W(e) + Lift(e~) + Pen_Y([h])
//     where W(v)[c] = sum_{a,d} eps_dac D_a v_d is the weak reference curl
//     (D_a[l][m] = (d_a phi_l, phi_m), [KS eq. matrix_free_curl]; the H equation
//     is used in its integrated-by-parts form, algebraically identical to the
//     strong form of [KS eq. cwc] for polynomial fields), s = sign(det A).
//     Part q traces and fluxes one face of the element and owns a quarter of
//     the output modes (volume rows, lift rows, mass inverse, PML, epilogue).
//     Leap-frog half steps give all lanes to the active field (four per
//     element).
//   * Reference matrices are compile-time constants (generated header): every
//     multiply by a structural zero disappears and every nonzero becomes an FMA
//     with an inline constant (p = 3: 202 of 1200 curl entries, 337 of 800
//     trace entries are nonzero). At ~2 flop/B the stage is bound by HBM; a
//     BF16x3 split-product MFMA form of the volume term is built as an option.
//   * Data movement per tile: the input fields are copied into LDS by
//     asynchronous buffer-to-LDS loads, together with the tile's halo block
//     and the RK operands, before the first barrier. Every lane traces its
//     input field on its face, tau_k(v)[m] = sum_l T_f[m][l] (v . t^_k)[l],
//     into an LDS slot. A face whose neighbour lies in another tile reads
//     the neighbour's traces from the halo block, which the neighbour's tile
//     wrote at the end of the previous launch: after its epilogue a tile
//     stages its output in LDS, traces it on those faces and stores the
//     traces into the reading tile's block of a global halo buffer. Both
//     elements of a face parametrise it from the face's vertices in
//     ascending global id, so traces combine without permutation;
//     the tangential cross product of [KS eqs. uwc/cwc] reduces to
//     int_F (a x n).b dS = sigma int (a.t2)(b.t1) - (a.t1)(b.t2) ds with
//     a.t_k = a^.t^_k for covariant fields and sigma = s sigma^_f.
//   * Upwind penalty: int_F [e]_t . v dS = sum_kl W_kl ([e].t_k)(v.t_l) with
//     W = sqrt(det g^) g^^-1, g^_kl = t^_k^T G0^-1 t^_l (G0^-1 = A^T A/|det A|).
//   * Mass inverse [KS Sec. III]: d_t u_l = (1/eps) G0^-1 r_l, 3x3 per mode.
//   * PML [KS Sec. IV, eqs. p_variable, q_variable] in Cartesian, eps-scaled
//     auxiliaries P~ = A^-T P / eps: d_t u = (1/eps) G0^-1 r - A^T(eta.c + P~),
//     d_t P~ = -w.P~ + xi.c, c = A^-T u.
//   * Tiles are mapped to workgroups XCD-major: consecutive tiles (spatial
//     neighbours) run on the same XCD and share its L2.
//
// This header holds the device code; stage_kernel.hip instantiates it for
// one (precision, order) pair per object (MDG_R, MDG_P), and stage_launch.hip
// dispatches to those instances.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "refops_dev_gen.h"
#include "refops_gen.h"
#include "stage_args.hpp"

namespace mdg {

template <int P>
using Ops = ref::Ops<P>;

// ---- raw buffer access (gfx9 buffer descriptor, bounds-checked by hardware)
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// cache policy: CP_NT marks streaming data (read or written once per launch)
// as non-temporal, so that it does not push reused data (geometry, tables)
// out of L2
enum { CP_DEF = 0, CP_NT = 2 };
template <typename R, int CP = CP_DEF>
__device__ __forceinline__ R bld(Rsrc r, uint32_t vo, uint32_t so) {
  if constexpr (sizeof(R) == 4) return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, CP));
  else return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, CP));
}
template <typename R, int CP = CP_DEF>
__device__ __forceinline__ void bst(R v, Rsrc r, uint32_t vo, uint32_t so) {
  if constexpr (sizeof(R) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, vo, so, CP);
  else {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, CP);
  }
}
__device__ __forceinline__ int32_t bldi(Rsrc r, uint32_t vo, uint32_t so) {
  return (int32_t)__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
}
// wave-uniform read of a table that no kernel of the launch writes, through
// the scalar cache (a plain load after stores in the same loop would be a
// vector load, and waiting for it would wait for every copy in flight)
__device__ __forceinline__ int32_t uniform_ld(const int32_t* p, int i) {
  return ((const __attribute__((address_space(4))) int32_t*)p)[i];
}
// byte offset of element e's block origin in a blocked array with `rows` rows
// per element: ((e/64)*rows*64 + e%64) * size
__device__ __forceinline__ uint32_t blk_base(uint32_t e, uint32_t rows, uint32_t size) {
  return ((e >> 6) * rows * 64u + (e & 63u)) * size;
}
// Windows: a workgroup touches only the (at most two) 64-element blocks of
// its tile, so a per-element array is addressed through a descriptor based
// at the tile's first block (64-bit address arithmetic once per tile) with
// 32-bit offsets relative to it, and no array is limited to 4 GiB. `on`
// false gives a zero-length descriptor (loads return 0, stores are dropped).
// nblk: the array's blocks (every element array holds whole blocks). The
// range is computed in 32-bit arithmetic: a 64-bit comparison would be done
// in vector registers, and a descriptor there turns every access through it
// into a loop over the lanes' values.
__device__ __forceinline__ Rsrc win_rsrc(const void* p, uint32_t nblk, uint32_t b0, uint32_t block_bytes,
                                         bool on = true) {
  // the saturating subtraction and the fused 64-bit multiply-add have only
  // vector forms: both results are taken back to scalar registers
  const uint32_t left = b0 < nblk ? nblk - b0 : 0u;
  const uint32_t len = __builtin_amdgcn_readfirstlane((left < 2u ? left : 2u) * block_bytes);
  const uint64_t addr = reinterpret_cast<uint64_t>(p) + (uint64_t)b0 * block_bytes;
  // (readfirstlane returns a signed int: zero-extend each half)
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)addr);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(addr >> 32));
  return make_rsrc(reinterpret_cast<const void*>(hi << 32 | lo), on ? len : 0u);
}
// element e's block origin relative to block b0 of its window
__device__ __forceinline__ uint32_t blk_rel(uint32_t e, uint32_t b0, uint32_t rows, uint32_t size) {
  return (((e >> 6) - b0) * rows * 64u + (e & 63u)) * size;
}
// byte offset of row r inside a block
template <typename R>
__device__ __forceinline__ constexpr uint32_t rowb(int r) { return (uint32_t)r * 64u * (uint32_t)sizeof(R); }

// ---- face parametrisation constants (local face f opposite vertex f)
// tangents t^1 = v_b - v_a, t^2 = v_c - v_a of the ascending face vertices:
//   f=0: (-1,1,0),(-1,0,1)  f=1: (0,1,0),(0,0,1)  f=2: (1,0,0),(0,0,1)  f=3: (1,0,0),(0,1,0)
// reference sign sigma^_f = sign((t^1 x t^2) . n^_out) = (+,-,+,-)
template <int F, typename R>
__device__ __forceinline__ R tan0(R x, R y, R z) {
  if constexpr (F == 0) return y - x;
  else if constexpr (F == 1) return y;
  else return x;
}
template <int F, typename R>
__device__ __forceinline__ R tan1(R x, R y, R z) {
  if constexpr (F == 3) return y;
  else if constexpr (F == 0) return z - x;
  else return z;
}
template <int F>
constexpr int ref_sign() { return (F == 0 || F == 2) ? 1 : -1; }

template <int F, typename R>
__device__ __forceinline__ void add_lift(R& ax, R& ay, R& az, R L1, R L2) {
  if constexpr (F == 0) { ax -= L1 + L2; ay += L1; az += L2; }
  else if constexpr (F == 1) { ay += L1; az += L2; }
  else if constexpr (F == 2) { ax += L1; az += L2; }
  else { ax += L1; ay += L2; }
}

// metric of face F: g^_kl = t^_k^T G t^_l for symmetric G
template <int F, typename R>
__device__ __forceinline__ void face_metric(R gxx, R gxy, R gxz, R gyy, R gyz, R gzz, R& g11, R& g12,
                                            R& g22) {
  if constexpr (F == 0) {
    g11 = gxx - 2 * gxy + gyy;
    g22 = gxx - 2 * gxz + gzz;
    g12 = gxx - gxy - gxz + gyz;
  } else if constexpr (F == 1) {
    g11 = gyy; g22 = gzz; g12 = gyz;
  } else if constexpr (F == 2) {
    g11 = gxx; g22 = gzz; g12 = gxz;
  } else {
    g11 = gxx; g22 = gyy; g12 = gxy;
  }
}

// ---- reference-operator constants
// FP32: the constexpr values become instruction literals (v_fmac_f32 with an
// inline constant). FP64: VOP3 has no literal form, so the values are read from
// packed tables in constant memory (scalar loads, consumed in table order).
template <typename R, int P>
struct Cst;
template <int P>
struct Cst<float, P> {
  static __device__ __forceinline__ float tr(int f, int m, int l) { return (float)Ops<P>::T[f][m][l]; }
  static __device__ __forceinline__ float tc(int f, int m, int l) { return (float)Ops<P>::T[f][m][l]; }
  static __device__ __forceinline__ float d(int a, int l, int m) { return (float)Ops<P>::D[a][l][m]; }
};
template <int P>
__device__ __forceinline__ const double* tabTR();
template <int P>
__device__ __forceinline__ const double* tabTC();
template <int P>
__device__ __forceinline__ const double* tabD();
#define MDG_TABS(p)                                                                  \
  template <>                                                                        \
  __device__ __forceinline__ const double* tabTR<p>() { return mdg_TpR_##p; }        \
  template <>                                                                        \
  __device__ __forceinline__ const double* tabTC<p>() { return mdg_TpC_##p; }        \
  template <>                                                                        \
  __device__ __forceinline__ const double* tabD<p>() { return mdg_DpV_##p; }
MDG_TABS(1)
MDG_TABS(2)
MDG_TABS(3)
MDG_TABS(4)
#undef MDG_TABS
template <int P>
struct Cst<double, P> {
  static __device__ __forceinline__ double tr(int f, int m, int l) { return tabTR<P>()[Ops<P>::TiR[f][m][l]]; }
  static __device__ __forceinline__ double tc(int f, int m, int l) { return tabTC<P>()[Ops<P>::TiC[f][m][l]]; }
  static __device__ __forceinline__ double d(int a, int l, int m) { return tabD<P>()[Ops<P>::DiV[a][l][m]]; }
};

// traces of a vector coefficient field on face F: t0/t1 = T_F (v . t^1/2)
// v(c, l): coefficient l of component c (a register array or an LDS row);
// MI: the field's modes (the first MI of the basis, the others are zero)
template <int P, int F, typename R, int MI = Ops<P>::N, typename V>
__device__ __forceinline__ void face_trace(const V& v, R (&t0)[Ops<P>::NF], R (&t1)[Ops<P>::NF]) {
  constexpr int NF = Ops<P>::NF;
#pragma unroll
  for (int m = 0; m < NF; ++m) {
    R s0 = 0, s1 = 0;
    bool first = true;
#pragma unroll
    for (int l = 0; l < MI; ++l) {
      if (Ops<P>::T[F][m][l] != 0.0) {
        const R c = Cst<R, P>::tr(F, m, l);
        const R a = tan0<F, R>(v(0, l), v(1, l), v(2, l));
        const R b = tan1<F, R>(v(0, l), v(1, l), v(2, l));
        s0 = first ? c * a : fma(c, a, s0);
        s1 = first ? c * b : fma(c, b, s1);
        first = false;
      }
    }
    t0[m] = s0;
    t1[m] = s1;
  }
}

// ---- work split: every (element, role) is served by four lanes, one per
// "part" Q (wave-uniform). Part Q traces face Q and owns the modes
// l = Q*NQ + i (i < NQ, l < N) of the output: volume rows, lift rows, mass
// inverse, PML and epilogue.
template <int P>
constexpr int nq() { return (Ops<P>::N + 3) / 4; }
// Face of part q. The trace work of a face is set by the sparsity of T_F
// (face 0, the slanted one, is the densest, then faces 3, 2, 1) and the
// volume and lift work of a mode group grows with its modes' degree, so
// part q takes mode group q and the faces in the opposite order of cost:
// this evens out the VALU work of the waves that meet at each barrier.
constexpr int face_of(int q) { return q == 0 ? 0 : 4 - q; }
// a compile-time count passed through a generic lambda
template <int V>
struct IC {
  static constexpr int value = V;
};

// acc[j][i] += sum_m T_F[m][l] (t^1[j] A1[m] + t^2[j] A2[m]),  l = Q*QS + i
// (QS modes per part), for the output modes l < MO
template <int P, int F, int Q, typename R, int MO = Ops<P>::N, int QS = nq<P>()>
__device__ __forceinline__ void face_lift_q(const R (&A1)[Ops<P>::NF], const R (&A2)[Ops<P>::NF],
                                            R (&acc)[3][nq<P>()]) {
  constexpr int NF = Ops<P>::NF, NQ = nq<P>();
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int l = Q * QS + i;
    if (i >= QS || l >= MO) continue;
    R L1 = 0, L2 = 0;
    bool first = true;
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      if (Ops<P>::T[F][m][l] != 0.0) {
        const R c = Cst<R, P>::tc(F, m, l);
        L1 = first ? c * A1[m] : fma(c, A1[m], L1);
        L2 = first ? c * A2[m] : fma(c, A2[m], L2);
        first = false;
      }
    }
    if (!first) add_lift<F, R>(acc[0][i], acc[1][i], acc[2][i], L1, L2);
  }
}

// acc = gs * W(v) on the modes l = Q*QS + i of part Q (QS modes per part):
//   W[x] = D_z v_y - D_y v_z, W[y] = D_x v_z - D_z v_x, W[z] = D_y v_x - D_x v_y
// for the input modes m < MI and the output modes l < MO (the others get 0)
template <int P, int Q, typename R, int MI = Ops<P>::N, int MO = Ops<P>::N, int QS = nq<P>(), typename V>
__device__ __forceinline__ void volume_q(const V& v, R gs, R (&acc)[3][nq<P>()]) {
  constexpr int NQ = nq<P>();
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int l = Q * QS + i;
    R ax = 0, ay = 0, az = 0;
    if (i < QS && l < MO) {
#pragma unroll
      for (int m = 0; m < MI; ++m) {
        if (Ops<P>::D[0][l][m] != 0.0) {
          const R cx = Cst<R, P>::d(0, l, m);
          ay = fma(cx, v(2, m), ay);
          az = fma(-cx, v(1, m), az);
        }
        if (Ops<P>::D[1][l][m] != 0.0) {
          const R cy = Cst<R, P>::d(1, l, m);
          ax = fma(-cy, v(2, m), ax);
          az = fma(cy, v(0, m), az);
        }
        if (Ops<P>::D[2][l][m] != 0.0) {
          const R cz = Cst<R, P>::d(2, l, m);
          ax = fma(cz, v(1, m), ax);
          ay = fma(-cz, v(0, m), ay);
        }
      }
    }
    acc[0][i] = gs * ax;
    acc[1][i] = gs * ay;
    acc[2][i] = gs * az;
  }
}

// LDS trace storage, slot-major: slot s (one face of one element) holds
// [role][k][m] = 4 NF reals, padded to an odd stride so that consecutive lanes
// (consecutive slots) hit distinct banks. A lane keeps one base address per
// slot; role, k and m become immediate offsets.
// C (compact): leap-frog halves with one field per workgroup keep only that
// field's input traces in the in-tile slots (stride 2 NF + 1)
template <int NF, bool C = false>
constexpr int slot_stride() { return C ? 2 * NF + 1 : 4 * NF + 1; }
template <int NF, bool C = false>
__device__ __forceinline__ int lbase(int slot, int role) {
  return slot * slot_stride<NF, C>() + (C ? 0 : role * 2 * NF);
}
template <int NF>
constexpr int loff(int k, int m) { return k * NF + m; }
// halo slots (index 4 tile + h): hrr reals per slot and field, 16-byte
// aligned. The halo buffers hold one region per reading role (region r: the
// traces that the role-r lanes read), each a sequence of per-tile blocks of
// nh slots; the LDS halo area is [region 0 block][region 1 block], or only
// the block of the active role with four lanes per element
template <int NF, typename R>
constexpr int hrr() { return (2 * NF * (int)sizeof(R) + 15) / 16 * 16 / (int)sizeof(R); }
// LDS offset of field `role`'s traces in slot `slot` (in-tile or halo; nh:
// the tile's halo slots, hb: LDS offset of the halo area)
template <int NF, typename R, bool C = false>
__device__ __forceinline__ int slot_base(int slot, int role, int tile, int nh, int hb) {
  const int h = slot - 4 * tile;
  return h < 0 ? lbase<NF, C>(slot, role) : hb + ((C ? 0 : role * nh) + h) * hrr<NF, R>();
}
// stores the NV consecutive reals v at byte offset vo (16-byte aligned) of r
template <typename R, int NV>
__device__ __forceinline__ void bst_run(const R (&v)[NV], Rsrc r, uint32_t vo) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  constexpr int ND = NV * (int)sizeof(R) / 4;
  uint32_t w[ND];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    if constexpr (sizeof(R) == 4) {
      w[i] = __builtin_bit_cast(uint32_t, v[i]);
    } else {
      const u32x2 d = __builtin_bit_cast(u32x2, v[i]);
      w[2 * i] = d.x;
      w[2 * i + 1] = d.y;
    }
  }
#pragma unroll
  for (int i = 0; i + 4 <= ND; i += 4) {
    const u32x4 q = {w[i], w[i + 1], w[i + 2], w[i + 3]};
    __builtin_amdgcn_raw_buffer_store_b128(q, r, vo, (uint32_t)(4 * i), 0);
  }
  if constexpr (ND % 4 >= 2) {
    const u32x2 q = {w[ND / 4 * 4], w[ND / 4 * 4 + 1]};
    __builtin_amdgcn_raw_buffer_store_b64(q, r, vo, (uint32_t)(4 * (ND / 4 * 4)), 0);
  }
  if constexpr (ND % 2 == 1) __builtin_amdgcn_raw_buffer_store_b32(w[ND - 1], r, vo, (uint32_t)(4 * (ND - 1)), 0);
}

// components of a field that enter the tangential trace on face F
template <int F>
constexpr bool face_needs(int c) {
  return (F == 0) || (F == 1 && c != 0) || (F == 2 && c != 1) || (F == 3 && c != 2);
}

// trace of a field on face F from the LDS output staging [role][3N][tile],
// stored to its halo-buffer slot: [input role of the field][k][m]
// (MO: the field's modes)
template <int P, int F, typename R, int MO = Ops<P>::N>
__device__ __forceinline__ void publish_face(const R* stg, int sf, int role, int tile, int li, Rsrc rH, int code,
                                             int hreg) {
  constexpr int N = Ops<P>::N, NF = Ops<P>::NF;
  R w[3][MO];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int l = 0; l < MO; ++l) w[c][l] = face_needs<F>(c) ? stg[((sf * 3 + c) * N + l) * tile + li] : R(0);
  R t0[NF], t1[NF];
  face_trace<P, F, R, MO>([&](int c, int l) { return w[c][l]; }, t0, t1);
  // a field's traces feed the neighbour lanes of the other role (the region
  // of that role); the slot is 16-byte aligned, so it goes out in 16-byte stores
  const uint32_t base = (uint32_t)(code + (1 - role) * hreg) * (uint32_t)sizeof(R);
  R v[2 * NF];
#pragma unroll
  for (int m = 0; m < NF; ++m) {
    v[m] = t0[m];
    v[NF + m] = t1[m];
  }
  bst_run<R, 2 * NF>(v, rH, base);
}

// RK4 stage epilogue, one code path for every stage. The descriptors select
// the stage: a load through a zero-length descriptor returns 0 without memory
// traffic, a store through one is dropped.
//   stage 0:    ACC = b k,         Uout = y + c dt k        (a = 0)
//   stage 1,2:  ACC = a + b k,     Uout = y + c dt k
//   stage 3:    Uout = y + dt (a + b k)                     (ACC store dropped;
//               Uout is Y itself for the in-place step)
//   operator:   Uout = k                                    (y = a = 0, c dt = 1)
// With a K array (k_on) the stage derivative k itself is stored there too.
//   leap-frog half (stage 4: E, 5: H): Y = y + dt k for the active field, with
//               y taken from the staged input (the stage input is Y itself) or,
//               with four lanes per element, loaded like the RK4 operands
// y_staged: y comes from the staged input in leap-frog halves and stage 0
struct Epi {
  Rsrc y_rd, a_rd, a_wr, out_wr, k_wr;
  bool final_stage, k_on;
  double c_out;  // c_{i+1} dt, dt (final, leap-frog) or 1 (operator)
};
__device__ __forceinline__ Epi make_epi(int stage, const void* Y, const void* ACC, const void* Uout, const void* K,
                                        uint32_t nblk, uint32_t b0, uint32_t block_bytes, double bcoef,
                                        double cdt, double dt, bool y_staged) {
  Epi e;
  const bool op = stage < 0, lf = stage >= 4;
  e.final_stage = stage == 3;
  e.y_rd = win_rsrc(Y, nblk, b0, block_bytes, !(op || (y_staged && (lf || stage == 0))));
  e.a_rd = win_rsrc(ACC, nblk, b0, block_bytes, stage >= 1 && stage <= 3);
  e.a_wr = win_rsrc(ACC, nblk, b0, block_bytes, stage >= 0 && stage <= 2);
  e.out_wr = win_rsrc(lf ? Y : Uout, nblk, b0, block_bytes);
  e.k_on = K != nullptr;
  e.k_wr = win_rsrc(K, nblk, b0, block_bytes, e.k_on);
  e.c_out = op ? 1.0 : ((e.final_stage || lf) ? dt : cdt);
  (void)bcoef;
  return e;
}
template <typename R>
__device__ __forceinline__ void rk_store(const Epi& e, R k, uint32_t vo, uint32_t so, R b, R c_out, bool live) {
  const R y = bld<R, CP_NT>(e.y_rd, vo, so);
  const R a = bld<R, CP_NT>(e.a_rd, vo, so);
  const R acc = fma(b, k, a);
  if (live) {
    bst<R, CP_NT>(acc, e.a_wr, vo, so);
    bst<R, CP_NT>(fma(c_out, e.final_stage ? acc : k, y), e.out_wr, vo, so);
    if (e.k_on) bst<R, CP_NT>(k, e.k_wr, vo, so);
  }
}
// same with y and a loaded earlier; returns the value written to the output
// (the next stage input, or the new Y)
template <typename R>
__device__ __forceinline__ R rk_store_pre(const Epi& e, R k, R y, R a, uint32_t vo, uint32_t so, R b, R c_out,
                                          bool live) {
  const R acc = fma(b, k, a);
  const R out = fma(c_out, e.final_stage ? acc : k, y);
  if (live) {
    bst<R, CP_NT>(acc, e.a_wr, vo, so);
    bst<R, CP_NT>(out, e.out_wr, vo, so);
    if (e.k_on) bst<R, CP_NT>(k, e.k_wr, vo, so);
  }
  return out;
}

// metric of face F (runtime face index): g^_kl = t^_k^T G t^_l
template <typename R>
__device__ __forceinline__ void face_metric_rt(int F, R gxx, R gxy, R gxz, R gyy, R gyz, R gzz, R& g11,
                                               R& g12, R& g22) {
  const R m11[4] = {gxx - 2 * gxy + gyy, gyy, gxx, gxx};
  const R m22[4] = {gxx - 2 * gxz + gzz, gzz, gzz, gyy};
  const R m12[4] = {gxx - gxy - gxz + gyz, gyz, gxz, gxy};
  g11 = m11[F];
  g22 = m22[F];
  g12 = m12[F];
}

// flux coefficients of face F in the face basis: the lift of the face term
// is sum_m T_F[m][l] (t^1 A1[m] + t^2 A2[m]). No reference matrix enters, so
// the face index is a runtime (wave-uniform) value.
template <int P, bool UPW, typename R, bool C = false>
__device__ __forceinline__ void face_flux_coef(int F, const R* lds, int role, int tile, int li, int hn, int hb, int code, R g,
                                               R sgn, R wz, R Z, R gxx, R gxy, R gxz, R gyy, R gyz, R gzz,
                                               R (&A1)[Ops<P>::NF], R (&A2)[Ops<P>::NF]) {
  constexpr int NF = Ops<P>::NF;
  const int so = F * tile + li;
  // PEC faces (code < 0) read the own trace with the mirror factor:
  // input field h+ = h- (role 0) / e+_t = -e-_t (role 1), i.e. factor g;
  // output field: factor -g
  const bool has = code >= 0;
  const int sn = has ? code : so;
  const R fin = has ? R(1) : g;
  const R* own = lds + lbase<NF, C>(so, role);
  const R* nbr = lds + slot_base<NF, R, C>(sn, role, tile, hn, hb);
  const R om = role ? R(1) - wz : wz;  // own weight of the averaged input field
  const R rsign = (F == 0 || F == 2) ? R(1) : R(-1);  // sigma^_f = (+,-,+,-)
  const R c = -g * rsign * sgn;
#pragma unroll
  for (int m = 0; m < NF; ++m) {
    const R xm0 = own[loff<NF>(0, m)];
    const R xm1 = own[loff<NF>(1, m)];
    const R xp0 = fin * nbr[loff<NF>(0, m)];
    const R xp1 = fin * nbr[loff<NF>(1, m)];
    const R xw0 = fma(om, xm0 - xp0, xp0);
    const R xw1 = fma(om, xm1 - xp1, xp1);
    A1[m] = c * xw1;
    A2[m] = -c * xw0;
  }
  if constexpr (UPW) {
    const R* own_o = lds + lbase<NF, C>(so, 1 - role);
    const R* nbr_o = lds + slot_base<NF, R, C>(sn, 1 - role, tile, hn, hb);
    R g11, g12, g22;
    face_metric_rt<R>(F, gxx, gxy, gxz, gyy, gyz, gzz, g11, g12, g22);
    const R idet = R(1) / sqrt(g11 * g22 - g12 * g12);
    const R pen = role ? Z * (R(1) - wz) : wz / Z;  // 1/(Y-+Y+) or 1/(Z-+Z+)
    const R W11 = pen * g22 * idet, W12 = -pen * g12 * idet, W22 = pen * g11 * idet;
    const R fout = has ? R(1) : -g;  // jump of the lane's output field
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      const R ym0 = own_o[loff<NF>(0, m)];
      const R ym1 = own_o[loff<NF>(1, m)];
      const R j0 = fma(fout, nbr_o[loff<NF>(0, m)], -ym0);
      const R j1 = fma(fout, nbr_o[loff<NF>(1, m)], -ym1);
      A1[m] = fma(W11, j0, fma(W12, j1, A1[m]));
      A2[m] = fma(W12, j0, fma(W22, j1, A2[m]));
    }
  }
}

// lift of all four faces onto the modes of part Q (QS per part, l < MO);
// the flux coefficients of face F of this element were published in its
// slot F*tile + li
template <int P, int Q, typename R, bool C = false, int MO = Ops<P>::N, int QS = nq<P>()>
__device__ __forceinline__ void lift_all_q(const R* lds, int role, int tile, int li, R (&acc)[3][nq<P>()]) {
  constexpr int NF = Ops<P>::NF;
  if constexpr (MO <= Q * QS) return;  // no output mode in this part
#define MDG_LIFT_FACE(F)                                                   \
  {                                                                        \
    asm volatile("" ::: "memory");                                         \
    const R* s_ = lds + lbase<NF, C>((F) * tile + li, role);               \
    R A1[NF], A2[NF];                                                      \
    _Pragma("unroll") for (int m = 0; m < NF; ++m) {                       \
      A1[m] = s_[loff<NF>(0, m)];                                          \
      A2[m] = s_[loff<NF>(1, m)];                                          \
    }                                                                      \
    face_lift_q<P, F, Q, R, MO, QS>(A1, A2, acc);                          \
  }
  MDG_LIFT_FACE(0)
  MDG_LIFT_FACE(1)
  MDG_LIFT_FACE(2)
  MDG_LIFT_FACE(3)
#undef MDG_LIFT_FACE
}

// ---- BF16x3 MFMA form of the volume term (FP32 state, 64-element tiles)
// The weak reference curl W of a tile's input field is one product
// W[3N x 64] = Dbig[3N x 3N] V[3N x 64] over the tile's elements [KS Sec. III,
// eq. matrix_free_curl]. The wave of part Q computes the rows of its output
// modes (rho = c NQ + i, one 16-row M-tile) for the 64 elements (four 16-column
// N-tiles) with v_mfma_f32_16x16x32_bf16 over K = 3N input rows in steps of 32.
// Both operands are split exactly into bfloat16 parts (x = hi + mid + lo; the
// constant side at build time), and the six products down to order 2^-16 are
// accumulated in FP32, smallest first, which keeps FP32 accuracy. Operand
// layouts (lane l): A row l % 16, K entries 8 (l / 16) .. +7; B column l % 16,
// the same K entries; D column l % 16, rows 4 (l / 16) .. +3. A 4 x 4 block
// transpose across the 16-lane rows (two permlane32 and two permlane16 swaps
// per accumulator register) hands every lane the 16 rows of its own element.
typedef __bf16 mdg_bf16x8 __attribute__((ext_vector_type(8)));
typedef float mdg_f32x4 __attribute__((ext_vector_type(4)));
template <int P>
__device__ __forceinline__ const uint4* mfa_table();
template <>
__device__ __forceinline__ const uint4* mfa_table<1>() { return reinterpret_cast<const uint4*>(mdg_mfA_1); }
template <>
__device__ __forceinline__ const uint4* mfa_table<2>() { return reinterpret_cast<const uint4*>(mdg_mfA_2); }
template <>
__device__ __forceinline__ const uint4* mfa_table<3>() { return reinterpret_cast<const uint4*>(mdg_mfA_3); }

// hi + mid + lo = x exactly (each part rounded to nearest even in turn)
__device__ __forceinline__ void split_bf16x3(const float (&x)[8], mdg_bf16x8& hi, mdg_bf16x8& mid, mdg_bf16x8& lo) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const __bf16 h = (__bf16)x[t];
    const float r1 = x[t] - (float)h;
    const __bf16 m = (__bf16)r1;
    const float r2 = r1 - (float)m;
    hi[t] = h;
    mid[t] = m;
    lo[t] = (__bf16)r2;
  }
}

// acc = gs W(v) on the modes of part `part`; stg_in: the tile's staged input
// field [3N][64] (LDS)
template <int P>
__device__ __forceinline__ void volume_mfma(const float* stg_in, int part, float gs, float (&acc)[3][nq<P>()]) {
  constexpr int N = Ops<P>::N, NQ = nq<P>(), R3 = 3 * N, KS = (R3 + 31) / 32;
  static_assert(3 * NQ <= 16, "one M-tile per part (orders up to 3)");
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  const uint4* tab = mfa_table<P>();
  mdg_f32x4 Cacc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) Cacc[j] = mdg_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    mdg_bf16x8 A[3];
#pragma unroll
    for (int sp = 0; sp < 3; ++sp)
      A[sp] = __builtin_bit_cast(mdg_bf16x8, tab[((part * KS + ks) * 3 + sp) * 64 + lane]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float x[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = 32 * ks + 8 * grp + t;
        const float v = stg_in[(k < R3 ? k : R3 - 1) * 64 + 16 * j + col];
        x[t] = k < R3 ? v : 0.f;
      }
      mdg_bf16x8 bh, bm, bl;
      split_bf16x3(x, bh, bm, bl);
      mdg_f32x4 c = Cacc[j];
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], bm, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], bl, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], bm, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], bh, c, 0, 0, 0);
      Cacc[j] = c;
    }
  }
  // lane d = 16 j + r gets rows 4 k + i of element d from lane 16 k + r of N-tile j
  float rows[16];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // the elements go through plain floats: a bit cast applied to a vector
    // element expression reads element 0 with this toolchain
    const float f0 = Cacc[0][i], f1 = Cacc[1][i], f2 = Cacc[2][i], f3 = Cacc[3][i];
    const unsigned u0 = __float_as_uint(f0), u1 = __float_as_uint(f1), u2 = __float_as_uint(f2),
                   u3 = __float_as_uint(f3);
    const auto s02 = __builtin_amdgcn_permlane32_swap(u0, u2, false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(u1, u3, false, false);
    const auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
    const auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
    const unsigned y0 = s01[0], y1 = s01[1], y2 = s23[0], y3 = s23[1];
    rows[i] = __uint_as_float(y0);
    rows[4 + i] = __uint_as_float(y1);
    rows[8 + i] = __uint_as_float(y2);
    rows[12 + i] = __uint_as_float(y3);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < NQ; ++i) acc[c][i] = gs * rows[c * NQ + i];
}

// Occupancy: LDS (4 NF + 1 reals per element and face) admits 2 workgroups
// per CU; with 8 lanes per element that is 16 waves (FP32, tile 64) or 8
// waves (FP64, tile 32) per CU, so registers are capped at 128 / 256. At
// p = 4 FP32 (32-element tiles) LDS admits 3 workgroups (12 waves), so the
// cap is 168 registers: the tighter one only forced spills without adding a
// wave. (FP64 at p = 4 needs more than the 256 architectural registers.)
template <typename R, int P>
constexpr int waves_per_eu() { return sizeof(R) == 4 ? (P >= 4 ? 3 : 4) : 2; }
// instances whose workgroups may take several tiles (see stage_kernel)
template <typename R, int P>
constexpr bool persistent_kernel() { return sizeof(R) == 4 && P <= 3; }

#define MDG_SWITCH_Q(...)                     \
  switch (part) {                             \
    case 0: { constexpr int Q = 0; __VA_ARGS__; } break; \
    case 1: { constexpr int Q = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int Q = 2; __VA_ARGS__; } break; \
    default: { constexpr int Q = 3; __VA_ARGS__; } break; \
  }

// LF: leap-frog half steps (stage 4/5), central flux only; the RK4 and
// operator launches use LF = 0, for which every leap-frog branch folds away.
// LF = 1 keeps eight lanes per element (both roles, one of them idle);
// LF = 2 (64-element tiles) gives every lane to the active field: four lanes
// per element and compact slots, so that four workgroups share a CU.
// SIP: the symmetric interior penalty surface unknown h_s of every face
// (central flux): part Q of the E lanes adds h_s of face Q to the averaged h
// trace, part Q of the H lanes advances h_s of face Q from the jump of the e
// traces (one copy per element face; both sides compute the same update).
// MF: the volume term by BF16x3 MFMA products (FP32, RK4 and operator calls,
// 64-element tiles) instead of the sparse VALU contraction.
// MIX: mixed orders (e at order P, h at P-1): the state's h rows (and those
// of its auxiliary q) hold only the dim P_{P-1} modes of h.
template <typename R, int P, bool UPW, bool PML, int LF, bool SIP = false, bool MF = false, bool MIX = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(waves_per_eu<R, P>()))) void stage_kernel(
    DevArgs a) {
  static_assert(!(LF && UPW), "leap-frog halves need the central flux");
  static_assert(!(SIP && UPW), "the SIP unknown comes with the central flux");
  static_assert(!MF || (sizeof(R) == 4 && LF == 0 && P <= 3), "MFMA volume: FP32, RK4, orders 1-3");
  static_assert(!MIX || P >= 2, "mixed orders: e at order 2 or more");
  constexpr bool C = LF == 2;
  constexpr int N = Ops<P>::N, NF = Ops<P>::NF, R3 = 3 * Ops<P>::N, NQ = nq<P>();
  // several tiles per workgroup (FP32, orders 1-3): in a loop the compiler
  // keeps loop-invariant values in registers, which the FP64 constant tables
  // and the order-4 register budget cannot afford
  constexpr bool PERSIST = persistent_kernel<R, P>();
  constexpr int SS = slot_stride<NF, C>();
  constexpr uint32_t RS = sizeof(R);
  // modes of h per component in the state; rows of one element block (e
  // rows c N + l, then h rows 3N + c NHc + l) and bytes of one 64-element block
  constexpr int NHc = MIX ? Ops<(P > 1 ? P - 1 : 1)>::N : N;
  // modes per part of the output h with mixed orders: its NHc modes spread
  // over the four parts, so that no wave does two parts' work while another
  // idles (the MFMA volume term keeps the parts of the full order)
  constexpr int QSH = MIX && !MF ? (NHc + 3) / 4 : NQ;
  // FP64 RK4: the first stage takes y from the staged input (its input is Y)
  constexpr bool YS0 = sizeof(R) == 8 && LF == 0;
  constexpr uint32_t RB = 3u * (N + NHc);
  constexpr uint32_t SBLK = RB * 64u * RS;
  // an offset past any window: a load there reads 0 (rows of h that the
  // compact layout does not hold)
  constexpr uint32_t OOB = 0x40000000u;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  // Tiles -> workgroups, XCD-major (dispatch places block b on XCD b % 8): the
  // workgroups of XCD x take the contiguous tile range [x T8, (x+1) T8),
  // T8 = ceil(ntiles / 8), so spatially adjacent tiles share that XCD's L2.
  // Workgroup j of an XCD (nx per XCD) takes tiles j, j + nx, j + 2 nx, ... of
  // the range: one tile each when the grid covers every tile, several when
  // the grid holds only the resident workgroups (persistent launch).
  const int nb = gridDim.x, b = blockIdx.x;
  const int nx = nb >> 3, T8 = (a.ntiles + 7) >> 3;
  const int tend = min((b & 7) * T8 + T8, a.ntiles);
  int tl = (b & 7) * T8 + (b >> 3);
  if (tl >= tend) return;  // whole block leaves together
  // the step's clock advances once, from a launch that no other kernel of the
  // step overlaps (the amplitudes of this stage were evaluated before it)
  if (a.tick && b == 0 && threadIdx.x == 0) a.tick[1] = a.tick[1] + 1.0;
  // 8 lanes per element (2 roles x 4 parts), or 4 (the active role's parts)
  // (the tile comes from the arguments: blockDim is read with a vector load,
  // whose wait would also wait for every copy in flight)
  const int tile = a.tile;
  const uint32_t nwv = (uint32_t)((C ? 4 : 8) * tile) >> 6;  // waves of the workgroup
  // LDS layout (reals): the in-tile trace slots [0, 4 tile SS), in which the
  // publication stages the tile's output fields [0, ST); the tile's input
  // field(s) [SB, SB + ST) as [field][3N][tile]; the halo slots from HB on.
  // ST = (C ? 1 : 2) 3N tile. With SB >= ST (when LDS allows it at the same
  // occupancy) a tile's input is copied in while the previous tile of the
  // workgroup publishes; with SB = 0 it shares the trace area and is copied
  // at the start of the tile.
  const int ST = (C ? 1 : 2) * R3 * tile;
  const int SB = a.stg_base, HB = a.halo_base;
  const bool early = SB >= ST;
  // the launch arguments, read through the kernel-argument segment
  typedef __attribute__((address_space(4))) const DevArgs KArgs;
  typedef __attribute__((address_space(3))) unsigned char lds_byte;
  // lane -> (part, role, element of the tile); the lanes of one part are a
  // multiple of 64, so the part is uniform in a wave. Part q owns the modes
  // q NQ + i of the output and the traces and fluxes of face face_of(q).
  struct Lane {
    int part, role, li;
  };
  auto lane_of = [&](KArgs& A, int tid) {
    Lane L;
    L.part = __builtin_amdgcn_readfirstlane(tid / (C ? tile : 2 * tile));
    // four parts: with it the compiler drops the mode-range branches where
    // 4 NQ = N (orders 1 and 3), which would split the epilogue into blocks
    // whose merged wait counts drain every memory operation in flight
    __builtin_assume(L.part >= 0 && L.part < 4);
    const int rem = tid - L.part * (C ? tile : 2 * tile);
    L.role = C ? A.stage - 4 : (rem >= tile);
    L.li = rem - (C ? 0 : L.role * tile);
    return L;
  };

  // 1. the input field(s) of a tile (role r lanes read field 1 - r) into
  // [SB, SB + ST) with asynchronous LDS loads, 16 bytes per lane and 1 KiB per
  // wave instruction: a row of the tile is tile RS bytes of one 64-element
  // block row, and the staged rows are consecutive rows of the state block
  auto input_copy = [&](KArgs& A, int tid, int tix) {
    const int fst = C ? 1 - (A.stage - 4) : 0;  // first staged field
    const uint32_t e0 = (uint32_t)(A.elem_begin + tix * tile), b0 = e0 >> 6;
    const uint32_t rsh = __builtin_ctz((uint32_t)tile * RS);  // log2 of the row bytes
    const uint32_t nbytes = (uint32_t)ST * RS;
    // cache policy of the copies: the input is read once per launch; marking
    // it non-temporal pays in FP64 (measured: RK4 stages 5%, leap-frog halves
    // with the SIP unknown 9%), except in the four-lane leap-frog halves
    // without it (4% slower), and not in FP32 (3% slower)
    constexpr int DMA_CP = sizeof(R) == 8 && (!C || SIP) ? CP_NT : CP_DEF;
    const Rsrc rU = win_rsrc(A.Uin, A.nblk, b0, SBLK);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    lds_byte* dst = (lds_byte*)smem_raw + (uint32_t)SB * RS;
    // state row of staging row sr ([staged field][3N]); with mixed orders
    // the staging keeps N modes per component of h, the state only NHc: the
    // others are not copied (`zero`). Traces and the volume term read only
    // the modes a field has; the MFMA volume term reads whole blocks, so for
    // it those rows are cleared first, before any copy is in flight (an LDS
    // store after an asynchronous copy into LDS waits for that copy).
    auto src_row = [&](uint32_t sr, bool& zero) -> uint32_t {
      const uint32_t f = C ? (uint32_t)fst : sr / R3, r = C ? sr : sr - f * R3;
      if constexpr (MIX) {
        const uint32_t cc = r / N, l = r - cc * N;
        zero = f == 1 && l >= (uint32_t)NHc;
        return f ? R3 + cc * NHc + l : r;
      } else {
        zero = false;
        return f * R3 + r;
      }
    };
    if constexpr (MIX && MF) {
      for (uint32_t vo = (uint32_t)tid * 4u; vo < nbytes; vo += nwv * 256u) {
        bool zero;
        src_row(vo >> rsh, zero);
        if (zero) *reinterpret_cast<uint32_t*>(smem_raw + (uint32_t)SB * RS + vo) = 0u;
      }
    }
    if (e0 % (uint32_t)tile == 0) {
      // the tile lies in one 64-element block: 16 bytes per lane
      const uint32_t base = blk_rel(e0, b0, RB, RS);
      for (uint32_t c = wv; c * 1024u < nbytes; c += nwv) {
        const uint32_t vo = c * 1024u + (uint32_t)(tid & 63) * 16u;
        bool zero;
        const uint32_t src = base + src_row(vo >> rsh, zero) * rowb<R>(1) + (vo & ((1u << rsh) - 1u));
        if (vo < nbytes && !zero) __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, dst + c * 1024u, 16, src, 0, 0, DMA_CP);
      }
    } else {
      // a tile of the damped partition that straddles two blocks: 4 bytes
      // per lane, each addressed through its own element
      for (uint32_t c = wv; c * 256u < nbytes; c += nwv) {
        const uint32_t vo = c * 256u + (uint32_t)(tid & 63) * 4u;
        const uint32_t w = vo & ((1u << rsh) - 1u);
        bool zero;
        const uint32_t src = blk_rel(e0 + w / RS, b0, RB, RS) + src_row(vo >> rsh, zero) * rowb<R>(1) + w % RS;
        if (vo < nbytes && !zero) __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, dst + c * 256u, 4, src, 0, 0, DMA_CP);
      }
    }
  };
  // 3. halo: the traces of out-of-tile neighbours were written by those
  // neighbours in the previous stage, as an image of the tile's halo slots;
  // the block is copied into the halo area the same way
  auto halo_copy = [&](KArgs& A, int tid, int tg) {
    const int role = lane_of(A, tid).role;
    const int hoff = uniform_ld(A.halo_tile, 2 * tg), hcount = uniform_ld(A.halo_tile, 2 * tg + 1);
    // the tile's block in each region (hrr reals per slot: a multiple of 16 bytes)
    const uint32_t rb = (uint32_t)hcount * hrr<NF, R>() * RS, jump = (uint32_t)A.hreg * RS;
    const uint32_t nbytes = C ? rb : 2u * rb;
    const Rsrc rH = make_rsrc(A.hin, A.hbuf_bytes);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    lds_byte* dst = (lds_byte*)smem_raw + (uint32_t)HB * RS;
    for (uint32_t c = wv; c * 1024u < nbytes; c += nwv) {
      const uint32_t vo = c * 1024u + (uint32_t)(tid & 63) * 16u;
      const uint32_t src = C ? vo + (uint32_t)role * jump : (vo < rb ? vo : vo - rb + jump);
      if (vo < nbytes) __builtin_amdgcn_raw_ptr_buffer_load_lds(rH, dst + c * 1024u, 16, src, (uint32_t)hoff * RS, 0, 0);
    }
  };
  // Rows of a lane's output field (role r: e or h) and of its auxiliary:
  // component c, mode l at voffset base + out_v(r, c, l), soffset out_s(c, l).
  // Equal orders: the soffset carries the whole row (uniform). Mixed orders:
  // the h rows have their own stride, which depends on the lane's role, so
  // the row goes into the voffset, and the rows l >= NHc of h are absent
  // (loads there read 0, stores are dropped).
  auto out_v = [&](int r, int c, int l) -> uint32_t {
    if constexpr (MIX)
      return r ? (l < NHc ? (uint32_t)(R3 + c * NHc + l) * rowb<R>(1) : OOB) : (uint32_t)(c * N + l) * rowb<R>(1);
    else
      return (uint32_t)r * rowb<R>(R3);
  };
  auto out_s = [&](int c, int l) -> uint32_t { return MIX ? 0u : (uint32_t)(c * N + l) * rowb<R>(1); };
  auto out_ok = [&](int r, int l) -> bool { return !MIX || r == 0 || l < NHc; };
  // output mode of slot q of part pt for role r, or N where there is none
  auto mode_of = [&](int r, int pt, int q) -> int {
    const int qs = MIX && r == 1 ? QSH : NQ, l = pt * qs + q;
    return q < qs && l < (MIX && r == 1 ? NHc : N) ? l : N;
  };
  // 2. RK operands of the part's output rows (absent operands read as 0),
  // requested with the tile's copies so that their latency overlaps the
  // trace, volume and flux work. FP32 loads the accumulator after barrier 1,
  // which keeps the register budget at four waves per SIMD.
  R ypre[3][NQ], apre[3][NQ];
  auto load_operands = [&](KArgs& A, int tid, int tix) {
    const Lane L = lane_of(A, tid);
    const uint32_t b0 = (uint32_t)(A.elem_begin + tix * tile) >> 6;
    const uint32_t e = (uint32_t)(A.elem_begin + tix * tile + L.li);
    const uint32_t vo = blk_rel(e, b0, RB, RS);
    const Epi ef = make_epi(A.stage, A.Y, A.ACC, A.Uout, A.Kout, A.nblk, b0, SBLK, A.bcoef, A.cdt, A.dt, LF == 1 || YS0);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int l = min(mode_of(L.role, L.part, q), N - 1);
        const uint32_t v = vo + out_v(L.role, c, l), so = out_s(c, l);
        ypre[c][q] = bld<R, CP_NT>(ef.y_rd, v, so);
        if constexpr (sizeof(R) == 8) apre[c][q] = bld<R, CP_NT>(ef.a_rd, v, so);
      }
  };
  // everything a tile needs from memory before its first barrier; the
  // copies go first, so that a barrier waits for them but not for the
  // operand loads behind them
  // FP64 RK4 stages of undamped elements issue these requests at raised wave
  // priority: a starting workgroup's copies and loads then go out ahead of
  // the arithmetic of the workgroup beside it on the same SIMDs (1.4% per
  // upwind stage). Measured, it gains nothing in FP32 and costs 1-2% in the
  // PML variant and the leap-frog halves, which keep the default.
  constexpr bool PRIO = sizeof(R) == 8 && LF == 0 && !PML;
  auto prefetch = [&](KArgs& A, int tid, int tix, bool with_input) {
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
    if (with_input) input_copy(A, tid, tix);
    halo_copy(A, tid, A.tile_begin + tix);
    __builtin_amdgcn_sched_barrier(0);
    load_operands(A, tid, tix);
    if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
  };
  prefetch(*(KArgs*)__builtin_amdgcn_kernarg_segment_ptr(), (int)threadIdx.x, tl, true);

  for (;;) {
  // the launch arguments and the lane's indices are re-derived for every
  // tile, opaque to the compiler, so that nothing computed from them (buffer
  // descriptors, LDS and memory offsets) is held in registers across tiles
  KArgs* ap = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  int tid = threadIdx.x;
  asm volatile("" : "+s"(ap), "+v"(tid));
  KArgs& a = *ap;
  const Lane lane = lane_of(a, tid);
  const int part = lane.part, role = lane.role, li = lane.li;
  const int face = part ? 4 - part : 0;  // face_of(part)
  const int t = a.tile_begin + tl;
  const int tnext = tl + nx;
  const bool more = PERSIST && tnext < tend;
  const int start = a.elem_begin + tl * tile;
  const int cnt = min(tile, a.elem_end - start);
  // Lanes past the end of a partial tile compute on padding (arrays are padded
  // by a full tile) so that every load is unconditional and every lane meets
  // every barrier; their stores are suppressed.
  const bool live = li < cnt;
  const uint32_t el = (uint32_t)(start + li);
  const uint32_t b0 = (uint32_t)start >> 6;  // first block of the tile (windows of the element arrays)
  const Rsrc rU = win_rsrc(a.Uin, a.nblk, b0, SBLK);
  const Rsrc rG = win_rsrc(a.geo, a.nblk, b0, NGEO * 64u * RS);
  const uint32_t vout = blk_rel(el, b0, RB, RS);  // element's state block
  const uint32_t vgeo = blk_rel(el, b0, NGEO, RS);
  const Epi ef = make_epi(a.stage, a.Y, a.ACC, a.Uout, a.Kout, a.nblk, b0, SBLK, a.bcoef, a.cdt, a.dt, LF == 1 || YS0);
  const int hn = uniform_ld(a.halo_tile, 2 * t + 1);  // halo slots of this tile
  const int hb = HB;
  __syncthreads();  // B0: the tile's input field(s) and halo block are in LDS
  const R* stg = lds + SB;

  // leap-frog half, and the first RK4 stage in FP64: the stage input is the
  // state itself, so the own rows of the output field come from the staging
  // (no second read of Y: in FP64 the non-temporal copy leaves no copy of it
  // in L2; in FP32 the second read hits L2 and the LDS reads cost more). In
  // the leap-frog half only the lanes of the active field store and publish.
  // The other role's lanes run along and their results are dropped (skipping
  // their work gains
  // nothing: the launch is bound by the workgroup's chain of loads and
  // barriers, and with 32-element tiles the two roles share waves). With the
  // central flux the active field's derivative reads no trace of its own
  // field, which is what lets the halves share one halo buffer.
  const int lf = LF ? a.stage - 4 : -1;
  const bool wr = live && (!LF || lf == role);
  if (LF == 1 || (YS0 && a.stage == 0)) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        // (the staging does not hold the modes of h beyond its order)
        const int l = mode_of(role, part, q);
        ypre[c][q] = l < N ? stg[(role * R3 + c * N + l) * tile + li] : R(0);
      }
  }

  // 4. trace of the input field on the part's face and the volume term of the
  // part's modes, both reading the input field from the staging (not held in
  // registers, which keeps the register budget at five waves per SIMD)
  const R* vin_lds = stg + (C ? 0 : 1 - role) * R3 * tile + li;
  auto vl = [&](int c, int l) { return vin_lds[(c * N + l) * tile]; };
  const R g = role ? R(-1) : R(1);
  // sign(det A); the adjoint operator negates the skew part (volume curl and
  // the averaged face term), which both carry this factor
  const R sgn = (a.adj ? R(-1) : R(1)) * bld<R>(rG, vgeo, rowb<R>(G_SIGN));
  R acc[3][NQ];
  {
    R t0[NF], t1[NF];
    // MI, MO: modes of the input and of the output field
    auto trace_volume = [&](auto mi, auto mo, auto qs) {
      constexpr int MI = decltype(mi)::value, MO = decltype(mo)::value, QS = decltype(qs)::value;
      if constexpr (MF) {
        volume_mfma<P>(stg + (1 - role) * R3 * tile, part, g * sgn, acc);
        asm volatile("" ::: "memory");
        MDG_SWITCH_Q((face_trace<P, face_of(Q), R, MI>(vl, t0, t1)));
      } else {
        MDG_SWITCH_Q((face_trace<P, face_of(Q), R, MI>(vl, t0, t1)));
        asm volatile("" ::: "memory");  // the volume term reads the staging again
        MDG_SWITCH_Q((volume_q<P, Q, R, MI, MO, QS>(vl, g * sgn, acc)));
      }
    };
    // mixed orders: the E lanes read h (NHc modes), the H lanes write it
    if (MIX && role == 0) trace_volume(IC<NHc>{}, IC<N>{}, IC<NQ>{});
    else trace_volume(IC<N>{}, IC<NHc>{}, IC<QSH>{});
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int i = 0; i < NQ; ++i) asm volatile("" : "+v"(acc[c][i]));
    __syncthreads();  // B0': every lane has read the staging
    R* d = lds + lbase<NF, C>(face * tile + li, role);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      d[loff<NF>(0, m)] = t0[m];
      d[loff<NF>(1, m)] = t1[m];
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  // 6. geometry and connectivity of the part's face, loaded while waiting at the
  // barrier (the input field is dead here)
  const R gxx = bld<R>(rG, vgeo, rowb<R>(G_XX)), gxy = bld<R>(rG, vgeo, rowb<R>(G_XY));
  const R gxz = bld<R>(rG, vgeo, rowb<R>(G_XZ)), gyy = bld<R>(rG, vgeo, rowb<R>(G_YY));
  const R gyz = bld<R>(rG, vgeo, rowb<R>(G_YZ)), gzz = bld<R>(rG, vgeo, rowb<R>(G_ZZ));
  R Z = 1, wz = 0.5;  // central: plain average
  if constexpr (UPW) {
    Z = bld<R>(rG, vgeo, rowb<R>(G_Z));
    wz = bld<R>(rG, vgeo, rowb<R>(G_WZ0 + face));
  }
  R sipc = 0;  // alpha_F / mu_F of the face
  if constexpr (SIP) sipc = bld<R>(rG, vgeo, rowb<R>(G_SIP0 + face));
  const R ieps = bld<R>(rG, vgeo, rowb<R>(G_IEPS)), imu = bld<R>(rG, vgeo, rowb<R>(G_IMU));
  const Rsrc rN = win_rsrc(a.nbr, a.nblk, b0, 4u * 64u * 4u);
  const int code = bldi(rN, blk_rel(el, b0, 4, 4), (uint32_t)face * 256u);
  const Rsrc rPub = win_rsrc(a.pub, a.nblk, b0, 4u * 64u * 4u);
  const int pcode = bldi(rPub, blk_rel(el, b0, 4, 4), (uint32_t)face * 256u);

  __syncthreads();  // B1: traces of the tile and its halo are in LDS
  if constexpr (sizeof(R) == 4) {
    // FP32: the accumulator rows are loaded here, still ~5 us before the
    // epilogue, which keeps the register budget at five waves per SIMD
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int lc = min(mode_of(role, part, q), N - 1);
        apre[c][q] = bld<R, CP_NT>(ef.a_rd, vout + out_v(role, c, lc), out_s(c, lc));
      }
  }

  // 7. flux coefficients of the part's face
  {
    R A1[NF], A2[NF];
    face_flux_coef<P, UPW, R, C>(face, lds, role, tile, li, hn, hb, code, g, sgn, wz, Z, gxx, gxy, gxz, gyy, gyz,
                                 gzz, A1, A2);
    if constexpr (SIP) {
      // the face of this element: sig = sign((t^1 x t^2) . n_out), rows
      // (face, k, m) of the element's surface block
      const R sig = ((face == 0 || face == 2) ? R(1) : R(-1)) * sgn;
      const uint32_t vs = blk_rel(el, b0, 8 * NF, RS);
      const int srow = face * 2 * NF;
      if (role == 0) {
        // E: -(h_s x n, v)_F has the form of the averaged h term, so the
        // edge-tangent components of h_s add to the averaged traces
        const Rsrc rS = win_rsrc(a.sUin, a.nblk, b0, 8u * NF * 64u * RS, a.sip != 0);
#pragma unroll
        for (int m = 0; m < NF; ++m) {
          const R s0 = bld<R>(rS, vs, rowb<R>(srow + m));
          const R s1 = bld<R>(rS, vs, rowb<R>(srow + NF + m));
          A1[m] = fma(-sig, s1, A1[m]);
          A2[m] = fma(sig, s0, A2[m]);
        }
      } else {
        // h_s: (mu/alpha) sqrt(det g) g^-1 d_t S = [-sig D_2; sig D_1] with
        // D_k the face coefficients of (e- - e+) . t^k (e+ = 0 on PEC faces);
        // the physical metric g is |det A| g^, whose Jacobian cancels
        R g11, g12, g22;
        face_metric_rt<R>(face, gxx, gxy, gxz, gyy, gyz, gzz, g11, g12, g22);
        const R fs = sipc / sqrt(g11 * g22 - g12 * g12);
        const bool has = code >= 0;
        const R* own = lds + lbase<NF, C>(face * tile + li, 1);
        const R* nbr = lds + slot_base<NF, R, C>(has ? code : face * tile + li, 1, tile, hn, hb);
        const R hn = has ? R(1) : R(0);
        const Epi es = make_epi(a.stage, a.sY, a.sACC, a.sUout, a.sKout, a.sip ? a.nblk : 0u, b0, 8u * NF * 64u * RS, a.bcoef,
                                a.cdt, a.dt, false);
        const R cs = R(es.c_out), bs = R(a.bcoef);
#pragma unroll
        for (int m = 0; m < NF; ++m) {
          // with mixed orders h_s lives in the lower-order face space, whose
          // modes are the first nfh of this basis: the others get no derivative
          const R keep = m < a.nfh ? R(1) : R(0);
          const R d0 = keep * fma(-hn, nbr[loff<NF>(0, m)], own[loff<NF>(0, m)]);
          const R d1 = keep * fma(-hn, nbr[loff<NF>(1, m)], own[loff<NF>(1, m)]);
          const R v1 = -sig * d1, v2 = sig * d0;
          rk_store<R>(es, fs * fma(g11, v1, g12 * v2), vs, rowb<R>(srow + m), bs, cs, wr);
          rk_store<R>(es, fs * fma(g12, v1, g22 * v2), vs, rowb<R>(srow + NF + m), bs, cs, wr);
        }
      }
    }
    __syncthreads();  // B2: every flux read of this tile is done
    // publish the flux coefficients of the face in its own slot
    R* d = lds + lbase<NF, C>(face * tile + li, role);
#pragma unroll
    for (int m = 0; m < NF; ++m) {
      d[loff<NF>(0, m)] = A1[m];
      d[loff<NF>(1, m)] = A2[m];
    }
  }
  __syncthreads();  // B3

  // 8. lift of the four faces onto this part's modes
  if (MIX && role == 1) {
    MDG_SWITCH_Q((lift_all_q<P, Q, R, C, NHc, QSH>(lds, role, tile, li, acc)));
  } else {
    MDG_SWITCH_Q((lift_all_q<P, Q, R, C>(lds, role, tile, li, acc)));
  }

  // 9. point currents (E lanes): r_E -= g(t) phi_l(r0) (A^-1 d)_j, with the
  // amplitudes g(t) of the stage's time evaluated just before the launch
  if (a.has_src && role == 0) {
    const Rsrc rS = win_rsrc(a.srcid, a.nblk, b0, 64u * 4u);
    int d = bldi(rS, blk_rel(el, b0, 1, 4), 0);
    if (d >= 0) {
      const R* __restrict__ src = reinterpret_cast<const R*>(a.src);
      for (; d >= 0; d = a.srcnext[d]) {
        const R amp = R(a.srcamp[d]);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int l = part * NQ + q;
            if (l < N) acc[c][q] = fma(-amp, src[(d * 3 + c) * N + l], acc[c][q]);
          }
      }
    }
  }

  // 10. 3x3 block-diagonal mass inverse: d_t u_l = (1/eps) G0^-1 r_l
  const R mf = role ? imu : ieps;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const R x = acc[0][q], y = acc[1][q], z = acc[2][q];
    acc[0][q] = mf * fma(gxx, x, fma(gxy, y, gxz * z));
    acc[1][q] = mf * fma(gxy, x, fma(gyy, y, gyz * z));
    acc[2][q] = mf * fma(gxz, x, fma(gyz, y, gzz * z));
  }

  // mixed orders: h lives in the lower-order space, whose modes are the first
  // NHc of this basis; its other modes get no derivative, so that they stay
  // zero in the output (the state does not hold them, but the traces that
  // the tile publishes are taken from the whole output), and the PML terms
  // below leave them at zero too
  if (MIX && role == 1) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (mode_of(1, part, q) >= N) acc[0][q] = acc[1][q] = acc[2][q] = R(0);
  }

  const R bc = R(a.bcoef);
  const int stage = a.stage;
  // rows of this part: row(c, q) = c*N + mode_of(role, part, q), skipped at N
  // 11. PML auxiliaries
  if constexpr (PML) {
    // damped elements are numbered from pml_base in the auxiliary arrays,
    // where the partition's tiles start at multiples of the tile
    const uint32_t pk = (uint32_t)((int64_t)el - a.pml_base);
    const uint32_t pb0 = (uint32_t)((int64_t)start - a.pml_base) >> 6;
    const Rsrc rP = win_rsrc(a.pml, a.pnblk, pb0, NPML * 64u * RS);
    const uint32_t vp = blk_rel(pk, pb0, NPML, RS);
    const Rsrc raU = win_rsrc(a.aUin, a.pnblk, pb0, SBLK);
    const Epi ea = make_epi(stage, a.aY, a.aACC, a.aUout, a.aKout, a.pnblk, pb0, SBLK, a.bcoef, a.cdt, a.dt, false);
    const R ca = R(ea.c_out);
    const uint32_t va = blk_rel(pk, pb0, RB, RS);
    R AT[9], AiT[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      AT[i] = bld<R>(rP, vp, rowb<R>(PM_AT + i));
      AiT[i] = bld<R>(rP, vp, rowb<R>(PM_AIT + i));
    }
    const R wx = bld<R>(rP, vp, rowb<R>(PM_OM + 0));
    const R wy = bld<R>(rP, vp, rowb<R>(PM_OM + 1));
    const R wzz = bld<R>(rP, vp, rowb<R>(PM_OM + 2));
    const R ex = wy + wzz - wx, ey = wzz + wx - wy, ez = wx + wy - wzz;
    const R xx = (wx - wy) * (wx - wzz), xy = (wy - wzz) * (wy - wx), xz = (wzz - wx) * (wzz - wy);
    // couplings u <- -q and q <- xi c; the adjoint in the mass inner product
    // (auxiliary weighted like its field, in Cartesian components) swaps
    // them: u <- xi q and q <- -c (the eta and w terms are self-adjoint)
    const R ux = a.adj ? -xx : R(1), uy = a.adj ? -xy : R(1), uz = a.adj ? -xz : R(1);
    const R qx = a.adj ? R(-1) : xx, qy = a.adj ? R(-1) : xy, qz = a.adj ? R(-1) : xz;
    const Rsrc raW = win_rsrc(a.aYw, a.pnblk, pb0, SBLK, LF != 0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int l = mode_of(role, part, q);
      if (l >= N) continue;
      R u[3], qa[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        u[c] = bld<R>(rU, vout + out_v(role, c, l), out_s(c, l));  // own output field at the stage input
        qa[c] = bld<R>(raU, va + out_v(role, c, l), out_s(c, l));
      }
      const R cx = AiT[0] * u[0] + AiT[1] * u[1] + AiT[2] * u[2];
      const R cy = AiT[3] * u[0] + AiT[4] * u[1] + AiT[5] * u[2];
      const R cz = AiT[6] * u[0] + AiT[7] * u[1] + AiT[8] * u[2];
      if (LF) {
        // leap-frog half with the damping terms by the trapezoid rule: per
        // Cartesian component, with k the undamped derivative and h = dt/2,
        //   x - c = dt k - h eta (x + c) - h (y + a),  y - a = h xi (x + c) - h w (y + a)
        // for the new field x and auxiliary y, solved exactly (2x2)
        const R h = R(0.5) * R(a.dt), dtr = R(a.dt);
        const R kc[3] = {AiT[0] * acc[0][q] + AiT[1] * acc[1][q] + AiT[2] * acc[2][q],
                         AiT[3] * acc[0][q] + AiT[4] * acc[1][q] + AiT[5] * acc[2][q],
                         AiT[6] * acc[0][q] + AiT[7] * acc[1][q] + AiT[8] * acc[2][q]};
        const R cc[3] = {cx, cy, cz}, et[3] = {ex, ey, ez}, xs[3] = {xx, xy, xz}, wv[3] = {wx, wy, wzz};
        R xn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const R b1 = fma(dtr, kc[c], fma(-h, fma(et[c], cc[c], qa[c]), cc[c]));
          const R b2 = fma(h, fma(xs[c], cc[c], -wv[c] * qa[c]), qa[c]);
          const R p1 = fma(h, et[c], R(1)), p2 = fma(h, wv[c], R(1));
          const R idet = R(1) / fma(h * h, xs[c], p1 * p2);
          xn[c] = (p2 * b1 - h * b2) * idet;
          const R yn = fma(p1, b2, h * xs[c] * b1) * idet;
          if (wr && out_ok(role, l)) bst<R, CP_NT>(yn, raW, va + out_v(role, c, l), out_s(c, l));
        }
        // the new covariant field, stored as is by the epilogue
        acc[0][q] = AT[0] * xn[0] + AT[1] * xn[1] + AT[2] * xn[2];
        acc[1][q] = AT[3] * xn[0] + AT[4] * xn[1] + AT[5] * xn[2];
        acc[2][q] = AT[6] * xn[0] + AT[7] * xn[1] + AT[8] * xn[2];
        continue;
      }
      const R y0 = fma(ex, cx, ux * qa[0]), y1 = fma(ey, cy, uy * qa[1]), y2 = fma(ez, cz, uz * qa[2]);
      acc[0][q] -= AT[0] * y0 + AT[1] * y1 + AT[2] * y2;
      acc[1][q] -= AT[3] * y0 + AT[4] * y1 + AT[5] * y2;
      acc[2][q] -= AT[6] * y0 + AT[7] * y1 + AT[8] * y2;
      const R k[3] = {fma(qx, cx, -wx * qa[0]), fma(qy, cy, -wy * qa[1]), fma(qz, cz, -wzz * qa[2])};
#pragma unroll
      for (int c = 0; c < 3; ++c)
        rk_store<R>(ea, k[c], va + out_v(role, c, l), out_s(c, l), bc, ca, live && out_ok(role, l));
    }
  }

  // 12. RK4 epilogue of this part's rows of the output field; acc becomes
  // the stored output
  {
    const R cf = R(ef.c_out);
    const bool direct = PML && LF;  // the PML block computed the new field
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int l = mode_of(role, part, q);
        if (l >= N) continue;
        const uint32_t v = vout + out_v(role, c, l), so = out_s(c, l);
        const bool ok = wr && out_ok(role, l);
        if (direct) {
          if (ok) bst<R, CP_NT>(acc[c][q], ef.out_wr, v, so);
        } else {
          acc[c][q] = rk_store_pre<R>(ef, acc[c][q], ypre[c][q], apre[c][q], v, so, bc, cf, ok);
        }
      }
  }

  // 13. traces of the output on faces that a neighbouring tile reads in the
  // next stage: stage the tile's output fields in LDS, then part Q traces
  // face face_of(Q) of its element into the neighbour tile's halo block. The next
  // tile's copies and operands are requested after the last barrier before
  // the final LDS reads of this tile.
  // the output is staged at OB: beside the trace slots when LDS has room
  // (one tile per workgroup), else in the trace area once the lifts are done
  const int OB = a.out_base;
  if (OB == 0) __syncthreads();  // B4: the lifts are done with the trace area
  const int sf = C ? 0 : role;
  if (a.publish) {
    R* sto = lds + OB;  // [role][3N][tile] ([active field][3N][tile] with four lanes per element)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int l = mode_of(role, part, q);
        if (l < N) sto[((sf * 3 + c) * N + l) * tile + li] = acc[c][q];
      }
    __syncthreads();  // B5
  }
  // the next tile's copies and operand loads; the first barrier of a tile
  // waits for all but the operand loads, so the copies must be issued before
  // those on every path into it
  if (more) {
    if (early) prefetch(a, tid, tnext, true);
    else halo_copy(a, tid, a.tile_begin + tnext);
  }
  if (a.publish && wr && pcode >= 0) {
    const Rsrc rHo = make_rsrc(a.hout, a.hbuf_bytes);
    if (MIX && role == 1) {
      MDG_SWITCH_Q((publish_face<P, face_of(Q), R, NHc>(lds + OB, sf, role, tile, li, rHo, pcode, a.hreg)));
    } else {
      MDG_SWITCH_Q((publish_face<P, face_of(Q), R>(lds + OB, sf, role, tile, li, rHo, pcode, a.hreg)));
    }
  }
  if (!more) break;
  tl = tnext;
  // without room for the next tile's input beside the output staging it is
  // copied now, once every lane has read the staging (B6), and the operand
  // loads follow it
  if (!early) {
    __syncthreads();  // B6
    input_copy(a, tid, tl);
    __builtin_amdgcn_sched_barrier(0);
    load_operands(a, tid, tl);
  }
  }  // tile loop
}
#undef MDG_SWITCH_Q


// ---------------------------------------------------------------- energy
// W = 1/2 sum_T sum_l eps u_l^T M u_l + mu f_l^T M f_l, M = (G0^-1)^-1 = |det A| A^-1 A^-T
template <typename R, int N>
__global__ __launch_bounds__(256) void energy_kernel(const R* __restrict__ Y, const R* __restrict__ geo, int64_t K,
                                                     double* __restrict__ part, double* __restrict__ eelem, int nh) {
  __shared__ double red[4];
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double w = 0.0;
  if (k < K) {
    const R* gk = geo + (k >> 6) * NGEO * 64 + (k & 63);
    const double a = gk[G_XX * 64], b = gk[G_XY * 64], c = gk[G_XZ * 64];
    const double d = gk[G_YY * 64], e = gk[G_YZ * 64], f = gk[G_ZZ * 64];
    const double det = a * (d * f - e * e) - b * (b * f - e * c) + c * (b * e - d * c);
    const double id = 1.0 / det;
    const double m00 = (d * f - e * e) * id, m01 = (c * e - b * f) * id, m02 = (b * e - c * d) * id;
    const double m11 = (a * f - c * c) * id, m12 = (b * c - a * e) * id, m22 = (a * d - b * b) * id;
    const double eps = 1.0 / (double)gk[G_IEPS * 64], mu = 1.0 / (double)gk[G_IMU * 64];
    // e rows c N + l, then h rows 3N + c nh + l (nh modes of h)
    const R* yk = Y + (k >> 6) * (int64_t)(3 * (N + nh)) * 64 + (k & 63);
    double sf[2] = {0.0, 0.0};
    for (int fld = 0; fld < 2; ++fld)
      for (int l = 0; l < (fld ? nh : N); ++l) {
        const int st = fld ? nh : N, b = fld * 3 * N;
        const double x = yk[(b + 0 * st + l) * 64];
        const double y = yk[(b + 1 * st + l) * 64];
        const double z = yk[(b + 2 * st + l) * 64];
        sf[fld] += m00 * x * x + m11 * y * y + m22 * z * z + 2.0 * (m01 * x * y + m02 * x * z + m12 * y * z);
      }
    w = 0.5 * (eps * sf[0] + mu * sf[1]);
    eelem[k] = w;
  }
  for (int o = 32; o > 0; o >>= 1) w += __shfl_down(w, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
// ---------------------------------------------------------------- publish
// Halo traces of a state set from the host (the stage kernels publish those
// of their own outputs): one lane per element and field, every face with a
// cross-tile neighbour.
template <int P, int F, typename R>
__device__ __forceinline__ void publish_face_global(const R (&w)[3][Ops<P>::N], int fld, Rsrc rH, int code,
                                                    int hreg) {
  constexpr int NF = Ops<P>::NF;
  R t0[NF], t1[NF];
  face_trace<P, F, R>([&](int c, int l) { return w[c][l]; }, t0, t1);
  const uint32_t base = (uint32_t)(code + (1 - fld) * hreg) * (uint32_t)sizeof(R);
#pragma unroll
  for (int m = 0; m < NF; ++m) {
    bst<R>(t0[m], rH, base, (uint32_t)(m * sizeof(R)));
    bst<R>(t1[m], rH, base, (uint32_t)((NF + m) * sizeof(R)));
  }
}

template <typename R, int P>
// (list non-null: only the listed elements, one per workgroup of 64 lanes)
__global__ __launch_bounds__(256) void publish_kernel(const void* U, uint32_t nblk, int nh, const int32_t* pub,
                                                      void* H, uint32_t hbuf_bytes, int K, int hreg,
                                                      const int64_t* list) {
  constexpr int N = Ops<P>::N, R3 = 3 * N;
  constexpr uint32_t RS = sizeof(R);
  int el, fld;
  uint32_t b0;  // windows at the block of the wave's elements
  if (list) {
    if (threadIdx.x >= 2) return;  // lanes 0, 1: the element's two fields
    el = (int)list[blockIdx.x];
    fld = (int)threadIdx.x;
    b0 = (uint32_t)el >> 6;
  } else {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    el = gid >> 1;
    fld = gid & 1;
    if (el >= K) return;
    // the 32 elements of a wave lie in one 64-element block
    b0 = (uint32_t)((blockIdx.x * 256 + (threadIdx.x & ~63u)) >> 1) >> 6;
  }
  const uint32_t rb = 3u * (uint32_t)(N + nh);  // rows of an element block: e, then h with nh modes
  const Rsrc rU = win_rsrc(U, nblk, b0, rb * 64u * RS), rP = win_rsrc(pub, nblk, b0, 4u * 64u * 4u);
  const Rsrc rH = make_rsrc(H, hbuf_bytes);
  const uint32_t vo = blk_rel((uint32_t)el, b0, rb, RS) + (uint32_t)fld * rowb<R>(R3);
  const int st = fld ? nh : N;  // row stride of the field's components
  int code[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) code[f] = bldi(rP, blk_rel((uint32_t)el, b0, 4, 4), (uint32_t)f * 256u);
  if (code[0] < 0 && code[1] < 0 && code[2] < 0 && code[3] < 0) return;
  R w[3][N];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int l = 0; l < N; ++l) w[c][l] = l < st ? bld<R>(rU, vo, rowb<R>(c * st + l)) : R(0);
  if (code[0] >= 0) publish_face_global<P, 0, R>(w, fld, rH, code[0], hreg);
  if (code[1] >= 0) publish_face_global<P, 1, R>(w, fld, rH, code[1], hreg);
  if (code[2] >= 0) publish_face_global<P, 2, R>(w, fld, rH, code[2], hreg);
  if (code[3] >= 0) publish_face_global<P, 3, R>(w, fld, rH, code[3], hreg);
}

// ------------------------------------------------- adjoint, upwind flux
// The upwind face terms depend on eps through the impedances Z = sqrt(mu/eps)
// of the two elements of a face: the own weight of the averaged input field
// (E rows: Z-/(Z- + Z+), H rows: Z+/(Z- + Z+)) and the penalty factor (E rows:
// 1/(Z- + Z+), H rows: Z- Z+/(Z- + Z+)); PEC faces mirror the element (weights
// 1/2, penalties 1/(2 Z) and Z/2). For the discrete adjoint, g_T gets
// dZ_T/deps_T times the derivative by Z_T of (a, A x) over the faces of T: the
// face terms of T's own equations and those of its neighbours' equations, for
// both fields. A x is the stage derivative before the mass inverse, a the
// adjoint stage vector, x the stage input; in the face basis (a, face term)
// = sum_m tau_1(a)[m] A1[m] + tau_2(a)[m] A2[m] (the lift is the transposed
// trace). Runs in FP64 on either state precision.

// traces of field fld (0: E, 1: H) of element e of the state u + cs du (du
// may be null) on face F (runtime)
template <typename R, int P>
__device__ void traces_rt(const R* __restrict__ u, const R* __restrict__ du, double cs, int64_t e, int fld, int F,
                          double (&t0)[Ops<P>::NF], double (&t1)[Ops<P>::NF], int nh) {
  constexpr int N = Ops<P>::N;
  const int st = fld ? nh : N;  // e rows c N + l, then h rows 3N + c nh + l
  const int64_t o = (e >> 6) * (int64_t)(3 * (N + nh)) * 64 + (e & 63) + fld * 3 * N * 64;
  auto v = [&](int c, int l) {
    if (l >= st) return 0.0;
    const int64_t r = o + (c * st + l) * 64;
    return (double)u[r] + (du ? cs * (double)du[r] : 0.0);
  };
  switch (F) {
    case 0: face_trace<P, 0, double>(v, t0, t1); break;
    case 1: face_trace<P, 1, double>(v, t0, t1); break;
    case 2: face_trace<P, 2, double>(v, t0, t1); break;
    default: face_trace<P, 3, double>(v, t0, t1); break;
  }
}

// d/dZ of (a, A x) for the face terms of element e's equations on its face F
// whose other side is (en, fn) (PEC: en = e, fn = F), given dom / dpen, the
// derivatives of the own weight and of the penalty factor, for field role r
template <typename R, int P>
__device__ double upw_side(const R* __restrict__ a, const R* __restrict__ x, const R* __restrict__ dx, double cs,
                           const R* __restrict__ geo, int64_t e, int F, int64_t en, int fn, bool has, int r,
                           double dom, double dpen, int nh) {
  constexpr int NF = Ops<P>::NF;
  const double g = r ? -1.0 : 1.0;
  const double fin = has ? 1.0 : g, fout = has ? 1.0 : -g;  // PEC mirror of the input / output field
  const R* ge = geo + (e >> 6) * NGEO * 64 + (e & 63);
  const double rsign = (F == 0 || F == 2) ? 1.0 : -1.0;
  const double c = -g * rsign * (double)ge[G_SIGN * 64];
  double g11, g12, g22;
  face_metric_rt<double>(F, ge[G_XX * 64], ge[G_XY * 64], ge[G_XZ * 64], ge[G_YY * 64], ge[G_YZ * 64],
                         ge[G_ZZ * 64], g11, g12, g22);
  const double idet = 1.0 / sqrt(g11 * g22 - g12 * g12);
  const double W11 = g22 * idet, W12 = -g12 * idet, W22 = g11 * idet;
  double ta0[NF], ta1[NF], v0[NF], v1[NF];
  traces_rt<R, P>(a, nullptr, 0.0, e, r, F, ta0, ta1, nh);  // the adjoint of the output field
  double s_avg = 0.0, s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
  // averaged input field: d(A1, A2)/dom = c (xm1 - xp1, -(xm0 - xp0))
  traces_rt<R, P>(x, dx, cs, e, 1 - r, F, v0, v1, nh);
  for (int m = 0; m < NF; ++m) s_avg += ta0[m] * v1[m] - ta1[m] * v0[m];
  traces_rt<R, P>(x, dx, cs, en, 1 - r, fn, v0, v1, nh);
  for (int m = 0; m < NF; ++m) s_avg -= fin * (ta0[m] * v1[m] - ta1[m] * v0[m]);
  // penalty on the jump of the output field: d(A1, A2)/dpen = W (j0, j1)
  traces_rt<R, P>(x, dx, cs, en, r, fn, v0, v1, nh);
  for (int m = 0; m < NF; ++m) {
    s00 += fout * ta0[m] * v0[m];
    s01 += fout * ta0[m] * v1[m];
    s10 += fout * ta1[m] * v0[m];
    s11 += fout * ta1[m] * v1[m];
  }
  traces_rt<R, P>(x, dx, cs, e, r, F, v0, v1, nh);
  for (int m = 0; m < NF; ++m) {
    s00 -= ta0[m] * v0[m];
    s01 -= ta0[m] * v1[m];
    s10 -= ta1[m] * v0[m];
    s11 -= ta1[m] * v1[m];
  }
  return dom * c * s_avg + dpen * (W11 * s00 + W12 * s01 + W12 * s10 + W22 * s11);
}

template <typename R, int P>
__global__ __launch_bounds__(64) void grad_upw_kernel(double* __restrict__ gout, const R* __restrict__ a,
                                                      const R* __restrict__ x, const R* __restrict__ dx, double cs,
                                                      const R* __restrict__ geo, const int32_t* __restrict__ nbrg,
                                                      int64_t K, double scale, int nh) {
  const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (k >= K) return;
  const R* gk = geo + (k >> 6) * NGEO * 64 + (k & 63);
  const double Z = gk[G_Z * 64], eps = 1.0 / (double)gk[G_IEPS * 64];
  double sum = 0.0;
  for (int F = 0; F < 4; ++F) {
    const int code = nbrg[4 * k + F];
    const bool has = code >= 0;
    const int64_t kn = has ? code >> 2 : k;
    const int fn = has ? (code & 3) : F;
    const double Zn = has ? (double)geo[(kn >> 6) * NGEO * 64 + (kn & 63) + G_Z * 64] : Z;
    const double S = Z + Zn, S2 = S * S;
    for (int r = 0; r < 2; ++r) {
      // own equations: weight and penalty by Z_T (= Z-)
      double dom, dpen;
      if (has) {
        dom = r ? -Zn / S2 : Zn / S2;
        dpen = r ? Zn * Zn / S2 : -1.0 / S2;
      } else {
        dom = 0.0;
        dpen = r ? 0.5 : -0.5 / (Z * Z);
      }
      sum += upw_side<R, P>(a, x, dx, cs, geo, k, F, kn, fn, has, r, dom, dpen, nh);
      // the neighbour's equations, where T is the other side (Z_T = Z+)
      if (has) {
        const double dom2 = r ? Zn / S2 : -Zn / S2;
        const double dpen2 = r ? Zn * Zn / S2 : -1.0 / S2;
        sum += upw_side<R, P>(a, x, dx, cs, geo, kn, fn, k, F, true, r, dom2, dpen2, nh);
      }
    }
  }
  gout[k] += scale * (-0.5 * Z / eps * sum);  // dZ/deps = -Z / (2 eps)
}

// ---------------------------------------------------------------- launch
static inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw Error(MDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// resident workgroups of a kernel on the current device (its occupancy times
// the CU count), looked up once per kernel and device
static int resident_workgroups(const void* kern, int block, size_t lds, int* cache) {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 16) dev = 15;
  if (cache[dev] > 0) return cache[dev];
  int per_cu = 0, ncu = 0;
  hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds),
            "hipOccupancyMaxActiveBlocksPerMultiprocessor");
  hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");
  cache[dev] = std::max(1, per_cu) * std::max(1, ncu);
  return cache[dev];
}

// persist: a grid of the resident workgroups only (rounded down to whole
// XCDs), each looping over its share of the tiles; otherwise one workgroup
// per tile
template <typename R, int P, bool MIX, bool UPW, bool PML, int LF, bool SIP = false, bool MF = false>
static void launch_one(const DevArgs& a, int tile, size_t lds, bool persist, hipStream_t st) {
  const void* kern = reinterpret_cast<const void*>(&stage_kernel<R, P, UPW, PML, LF, SIP, MF, MIX>);
  const int block = (LF == 2 ? 4 : 8) * tile;
  if (lds > 64 * 1024)
    hip_check(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "hipFuncSetAttribute(dynamic LDS)");
  int grid = (a.ntiles + 7) / 8 * 8;
  DevArgs b = a;
  if (persist && persistent_kernel<R, P>()) {
    static int cache[16] = {0};
    const int res = resident_workgroups(kern, block, lds, cache);
    grid = std::min(grid, std::max(8, res / 8 * 8));
    // the next tile's copies land beside the trace slots while this tile
    // publishes, so the output is staged in the trace area
    b.out_base = 0;
  }
  hipLaunchKernelGGL((stage_kernel<R, P, UPW, PML, LF, SIP, MF, MIX>), dim3(grid), dim3(block), lds, st, b);
  hip_check(hipGetLastError(), "stage_kernel launch");
}

// RK4 stage or operator call with the MFMA volume term (FP32, orders 1-3, 64-element tiles)
template <typename R, int P, bool MIX>
static void launch_mfma(const DevArgs& a, bool upw, bool sip, bool pml, int tile, size_t lds, bool ps,
                        hipStream_t st) {
  if constexpr (sizeof(R) == 4 && P <= 3) {
    if (tile != 64) throw Error(MDG_E_UNSUPPORTED, "the MFMA volume term needs 64-element tiles");
    if (upw) {
      if (pml) launch_one<R, P, MIX, true, true, 0, false, true>(a, tile, lds, ps, st);
      else launch_one<R, P, MIX, true, false, 0, false, true>(a, tile, lds, ps, st);
    } else if (sip) {
      if (pml) launch_one<R, P, MIX, false, true, 0, true, true>(a, tile, lds, ps, st);
      else launch_one<R, P, MIX, false, false, 0, true, true>(a, tile, lds, ps, st);
    } else {
      if (pml) launch_one<R, P, MIX, false, true, 0, false, true>(a, tile, lds, ps, st);
      else launch_one<R, P, MIX, false, false, 0, false, true>(a, tile, lds, ps, st);
    }
  } else {
    throw Error(MDG_E_UNSUPPORTED, "the MFMA volume term is built for FP32 and orders 1-3");
  }
}

// central-flux launches with or without the SIP unknown
template <typename R, int P, bool MIX, bool PML, int LF>
static void launch_c(const DevArgs& a, bool sip, int tile, size_t lds, bool ps, hipStream_t st) {
  if (sip) launch_one<R, P, MIX, false, PML, LF, true>(a, tile, lds, ps, st);
  else launch_one<R, P, MIX, false, PML, LF, false>(a, tile, lds, ps, st);
}

template <typename R, int P, bool MIX>
static void launch_pm(const DevArgs& a, bool upw, bool sip, bool pml, int tile, size_t lds, bool mfma, bool ps,
                      hipStream_t st) {
  if (upw && sip) throw Error(MDG_E_UNSUPPORTED, "the SIP unknown needs the central flux");
  if (mfma) {
    if (a.stage >= 4) throw Error(MDG_E_UNSUPPORTED, "the MFMA volume term runs with RK4");
    launch_mfma<R, P, MIX>(a, upw, sip, pml, tile, lds, ps, st);
    return;
  }
  if (a.stage >= 4) {  // leap-frog half (central flux, checked at creation)
    if (upw) throw Error(MDG_E_UNSUPPORTED, "leap-frog needs the central flux");
    if (tile % 64 == 0) {  // four lanes per element
      if (pml) launch_c<R, P, MIX, true, 2>(a, sip, tile, lds, ps, st);
      else launch_c<R, P, MIX, false, 2>(a, sip, tile, lds, ps, st);
    } else {
      if (pml) launch_c<R, P, MIX, true, 1>(a, sip, tile, lds, ps, st);
      else launch_c<R, P, MIX, false, 1>(a, sip, tile, lds, ps, st);
    }
  } else if (upw) {
    if (pml) launch_one<R, P, MIX, true, true, 0>(a, tile, lds, ps, st);
    else launch_one<R, P, MIX, true, false, 0>(a, tile, lds, ps, st);
  } else {
    if (pml) launch_c<R, P, MIX, true, 0>(a, sip, tile, lds, ps, st);
    else launch_c<R, P, MIX, false, 0>(a, sip, tile, lds, ps, st);
  }
}

// mix: the state holds h (and q) with the modes of order P-1 only
template <typename R, int P>
void launch_p(const DevArgs& a, bool upw, bool sip, bool pml, int tile, size_t lds, bool mfma, bool ps, bool mix,
              hipStream_t st) {
  if (!mix) {
    launch_pm<R, P, false>(a, upw, sip, pml, tile, lds, mfma, ps, st);
  } else {
    if constexpr (P >= 2) launch_pm<R, P, true>(a, upw, sip, pml, tile, lds, mfma, ps, st);
    else throw Error(MDG_E_UNSUPPORTED, "mixed orders need e at order 2 or more");
  }
}

template <typename R, int P>
void launch_energy_rp(const void* Y, const void* geo, int64_t K, double* part, double* eelem, int nh, hipStream_t st) {
  const int64_t nblk = (K + 255) / 256;
  hipLaunchKernelGGL((energy_kernel<R, Ops<P>::N>), dim3(nblk), dim3(256), 0, st, static_cast<const R*>(Y),
                     static_cast<const R*>(geo), K, part, eelem, nh);
  hip_check(hipGetLastError(), "energy_kernel launch");
}

template <typename R, int P>
void launch_publish_rp(const void* U, uint32_t nblk, int nh, const int32_t* pub, void* H, uint32_t hb, int K,
                       int hreg, const int64_t* list, int nlist, hipStream_t st) {
  if (list) {
    if (nlist > 0)
      hipLaunchKernelGGL((publish_kernel<R, P>), dim3(nlist), dim3(64), 0, st, U, nblk, nh, pub, H, hb, K, hreg, list);
  } else {
    const dim3 grid((unsigned)((2 * (int64_t)K + 255) / 256));
    hipLaunchKernelGGL((publish_kernel<R, P>), grid, dim3(256), 0, st, U, nblk, nh, pub, H, hb, K, hreg, list);
  }
  hip_check(hipGetLastError(), "publish_kernel launch");
}

template <typename R, int P>
void launch_grad_upw_rp(double* g, const void* a, const void* x, const void* dx, double cs, const void* geo,
                        const int32_t* nbrg, int64_t K, double scale, int nh, hipStream_t st) {
  const dim3 grid((unsigned)((K + 63) / 64));
  hipLaunchKernelGGL((grad_upw_kernel<R, P>), grid, dim3(64), 0, st, g, static_cast<const R*>(a),
                     static_cast<const R*>(x), static_cast<const R*>(dx), cs, static_cast<const R*>(geo), nbrg, K,
                     scale, nh);
  hip_check(hipGetLastError(), "grad_upw_kernel launch");
}

}  // namespace mdg

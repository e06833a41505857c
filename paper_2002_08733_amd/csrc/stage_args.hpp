// stage_args.hpp -- the argument block of the stage kernel and the
// per-(precision, order) launchers that stage_kernel.hip instantiates and
// stage_launch.hip calls.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "solver.hpp"

namespace mdg {

struct DevArgs {
  const void* Y;      // RK base state u^n (E,H), blocked layout
  const void* Uin;    // stage input
  void* Uout;         // next stage input / operator output / new state (final stage)
  void* Kout;         // non-null: the stage derivative k is stored here too
  void* ACC;          // RK accumulator
  const void* aY;     // same for the PML auxiliaries
  const void* aUin;
  void* aUout;
  void* aKout;
  void* aACC;
  void* aYw;
  const void* sY;     // SIP surface unknown [K/64][face][k][NF][64]: RK base (leap-frog: updated in place)
  const void* sUin;   // stage input
  void* sUout;        // next stage input / operator output / new state (final stage)
  void* sKout;        // non-null: the stage derivative stored here too
  void* sACC;         // RK accumulator
  const void* geo;
  const int32_t* nbr;
  const int32_t* pub;        // publish codes: halo-buffer offset of each face's trace, or -1
  const int32_t* halo_tile;  // per tile: halo block offset (reals), halo slot count
  const void* hin;           // halo traces of the stage input
  void* hout;                // halo traces of the stage output
  const void* pml;
  const void* src;            // dipole load vectors [ndip][3][N]
  const int32_t* srcid;       // blocked [Kpad/64][64]: first dipole acting on the element, or -1
  const int32_t* srcnext;     // [ndip]: next dipole on the same element, or -1
  const double* srcamp;       // [ndip]: g(t) of every dipole at the launch's time
  double* tick;               // non-null: advance this device clock (n += 1) once
  // array sizes: the element arrays (whole 64-element blocks) are addressed
  // through per-tile windows and given in blocks (any size): nblk for the
  // arrays over all elements, pnblk for those over the damped ones; the halo
  // buffers through 32-bit offsets (under 4 GiB)
  uint32_t nblk, pnblk, hbuf_bytes;
  int32_t sip;  // the SIP surface arrays exist
  int64_t pml_base;
  int32_t tile_begin, ntiles, stage, has_src, publish;  // stage: 0..3 RK4, -1 operator, 4/5 leap-frog E/H half
  int32_t elem_begin, elem_end;  // element range of this launch (tiles of `tile` elements from elem_begin)
  int32_t nh;                    // modes of h: N, or fewer with mixed orders (the rest stay zero)
  int32_t nfh;                   // face modes of the SIP unknown: NF, or fewer with mixed orders
  int32_t hreg;                  // reals of one field's region of the halo buffers
  int32_t adj;                   // 1: adjoint operator (operator calls without sources)
  int32_t stg_base, halo_base;   // LDS offsets (reals) of the staged input and of the halo slots
  int32_t out_base;              // LDS offset (reals) of the output staging of the publication (0: the trace area)
  int32_t tile;                  // elements per workgroup (block: 8 lanes per element, 4 for compact leap-frog halves)
  double bcoef, cdt, dt;
};

template <typename R, int P>
void launch_p(const DevArgs& a, bool upw, bool sip, bool pml, int tile, size_t lds, bool mfma, bool persist,
              bool mix, hipStream_t st);
template <typename R, int P>
void launch_energy_rp(const void* Y, const void* geo, int64_t K, double* part, double* eelem, int nh, hipStream_t st);
template <typename R, int P>
void launch_publish_rp(const void* U, uint32_t nblk, int nh, const int32_t* pub, void* H, uint32_t hb, int K,
                       int hreg, const int64_t* list, int nlist, hipStream_t st);
template <typename R, int P>
void launch_grad_upw_rp(double* g, const void* a, const void* x, const void* dx, double cs, const void* geo,
                        const int32_t* nbrg, int64_t K, double scale, int nh, hipStream_t st);

// every (precision, order) pair the library is built for
#define MDG_FOR_EACH_RP(X) X(float, 1) X(float, 2) X(float, 3) X(float, 4) X(double, 1) X(double, 2) X(double, 3) X(double, 4)

}  // namespace mdg

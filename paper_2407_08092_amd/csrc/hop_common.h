// hop_common.h -- pieces shared by the stencil kernels: neighbour sites, one hop
// (spin projection, SU(3) multiply, reconstruction) and the load schedule.
#pragma once

#include "ddq_internal.h"

namespace ddq {

// neighbour sites of hop h (h = 2 mu + 0: forward x + mu, h = 2 mu + 1: backward
// x - mu) and the boundary sign of the t hops
struct Nbr {
  int j[8];
  float sgn_tf, sgn_tb;
};

__device__ __forceinline__ Nbr neighbours(const Geo& g, const Site& s) {
  Nbr n;
  {
    int base = s.i - (s.x >> 1);
    int xf = (s.x + 1 == g.L[0]) ? 0 : s.x + 1;
    int xb = (s.x == 0) ? g.L[0] - 1 : s.x - 1;
    n.j[0] = base + (xf >> 1);
    n.j[1] = base + (xb >> 1);
  }
  n.j[2] = (s.y + 1 == g.L[1]) ? s.i - (g.L[1] - 1) * g.sY : s.i + g.sY;
  n.j[3] = (s.y == 0) ? s.i + (g.L[1] - 1) * g.sY : s.i - g.sY;
  n.j[4] = (s.z + 1 == g.L[2]) ? s.i - (g.L[2] - 1) * g.sZ : s.i + g.sZ;
  n.j[5] = (s.z == 0) ? s.i + (g.L[2] - 1) * g.sZ : s.i - g.sZ;
  const bool wf = (s.t + 1 == g.L[3]), wb = (s.t == 0);
  n.j[6] = wf ? s.i - (g.L[3] - 1) * g.sT : s.i + g.sT;
  n.j[7] = wb ? s.i + (g.L[3] - 1) * g.sT : s.i - g.sT;
  n.sgn_tf = (g.antiperiodic && wf) ? -1.f : 1.f;
  n.sgn_tb = (g.antiperiodic && wb) ? -1.f : 1.f;
  return n;
}

template <typename R>
__device__ __forceinline__ void scale_half(Half<R>& h, R f) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) h.c[s][c] = f * h.c[s][c];
}

// Orders one hop before the next: the accumulator is routed through an empty
// volatile asm, so the hop's arithmetic has to finish here, and the memory
// clobber keeps later loads below.  Without it the instruction selector lifts
// all 96 neighbour loads to the top and spills them.
template <typename R>
__device__ __forceinline__ void hop_fence(Spinor<R>& acc) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc.c[sp][c].r), "+v"(acc.c[sp][c].i)::"memory");
  __builtin_amdgcn_sched_barrier(0);
}

// software pipelining: issue hop h+1's loads before hop h's arithmetic
#ifndef DDQ_PREFETCH
#define DDQ_PREFETCH 1
#endif

template <typename R>
struct HopCtx {
  Field in;
  const pair<R>* links;
  int lrows;      // complex rows of one direction's link field (18, or 12 with LINK12)
  int vh;
  uint32_t loff;  // lane offset of the output site in a link field
  Nbr nb;
  R sf, sb;       // projector signs of forward and backward hops
};

// link field of direction mu (LINK_ROWS complex rows, blocked)
template <typename R>
__device__ __forceinline__ Field link_field(const HopCtx<R>& c, int mu) {
  return bfield(c.links + (size_t)mu * c.lrows * field_vh(c.vh), c.lrows / CPE<R>, c.vh);
}

// acc += (1 + sg g_mu) U in(neighbour), hop H
template <int H, typename R>
__device__ __forceinline__ void hop_compute(Spinor<R>& acc, const Spinor<R>& p, const Link<R>& u,
                                            const HopCtx<R>& c) {
  constexpr int MU = H >> 1;
  const R sg = (H & 1) ? c.sb : c.sf;
  Half<R> h = project<MU, R>(p, sg);
  Half<R> uh = link_mul<R>(u, h);
  if (MU == 3) scale_half(uh, (R)((H & 1) ? c.nb.sgn_tb : c.nb.sgn_tf));
  accumulate<MU, R>(acc, uh, sg);
}

// Loads of hop H: the neighbour spinor, and the link.  FP64 reads one 9-entry half
// of a direction's link field per hop; FP32 reads both halves (nine 16-byte
// elements) at the forward hop and keeps the backward link for the next hop.
template <int H, typename R, bool L12>
__device__ __forceinline__ void hop_loads(const HopCtx<R>& c, Spinor<R>& p, Link<R>& u, Link<R>& u_bwd) {
  p = load_spinor<R>(c.in, voff(c.nb.j[H]));
  if constexpr (CPE<R> == 1 && !L12) {
    u = load_link_half<R>(link_field(c, H >> 1), H & 1, c.loff);
  } else if constexpr ((H & 1) == 0) {
    if constexpr (L12)
      load_link_pair12<R>(link_field(c, H >> 1), c.loff, u, u_bwd);
    else
      load_link_pair<R>(link_field(c, H >> 1), c.loff, u, u_bwd);
  } else {
    u = u_bwd;
    if constexpr (L12) su3_third_row(u);
  }
}

template <int H, typename R, bool L12>
__device__ __forceinline__ void hop_steps(Spinor<R>& acc, Spinor<R>& p, Link<R>& u, Link<R>& u_bwd,
                                          const HopCtx<R>& c) {
  if constexpr (DDQ_PREFETCH && H < 7) {
    Spinor<R> pn;
    Link<R> un, ub = u_bwd;
    hop_loads<H + 1, R, L12>(c, pn, un, ub);
    hop_compute<H, R>(acc, p, u, c);
    hop_fence<R>(acc);
    hop_steps<H + 1, R, L12>(acc, pn, un, ub, c);
  } else {
    hop_compute<H, R>(acc, p, u, c);
    hop_fence<R>(acc);
    if constexpr (H < 7) {
      Spinor<R> pn;
      Link<R> un, ub = u_bwd;
      hop_loads<H + 1, R, L12>(c, pn, un, ub);
      hop_steps<H + 1, R, L12>(acc, pn, un, ub, c);
    }
  }
}

}  // namespace ddq

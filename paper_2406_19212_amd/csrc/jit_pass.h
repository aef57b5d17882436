// Circuit-specialised fused passes (pure states, LDS tiles).
//
// The interpreting pass kernel (k_pass_lds) reads each op's kind and register
// bits from its program and branches to the matching code: about 40 scalar
// instructions and a few branches per op, next to 50-60 FP64 FMAs.  Here the
// host planner emits, for each pass of a circuit, a small description -- the
// tile's qubits, each stage's register bits and the kind and register bits of
// every op -- and this driver is compiled against it at run time (hipRTC).
// Every index of the tile, the stages and the ops is then a compile-time
// constant; only the op parameters (rotation records, matrix offsets) and the
// state pointers are read at run time, from the same op program and job
// tables the interpreter uses, and the same register-level op templates
// (pass_kernels.h) do the arithmetic.
//
// A pass description P provides
//   K, R                   tile bits and register bits
//   NST                    stages
//   TQ[K]                  physical bit of tile-local bit i (input layout)
//   TQO[K], LBO[K]         output layout: physical bits in ascending order and
//                          the tile-local bit stored at each
//   RBIT[NST][R]           tile-local bit held in register bit i of a stage
//   SRT[NST][R]            the same bits in ascending order
//   SWC[K]                 LDS bank swizzle: tile-local index l is kept at
//                          slot (l & ~15) | (XOR of SWC[q] over the set bits q
//                          of l), chosen by the planner for this pass's access
//                          patterns; SWB its width, SWDEF when it is the fixed
//                          fold l ^ ((l >> 4) ^ (l >> 8)) & 15
//   TAB                    offset of the pass's rows in the lane-slot table
//                          (a kernel argument)
//   DIN                    the first stage holds none of the low bits: it
//                          reads HBM directly
//   DOUT                   the last stage's wave lanes cover the output's low
//                          bits: it stores straight to HBM
//   MOVES, TQL[K]          the output layout differs from the input's; output
//                          physical bit of tile-local bit i
//   NH                     ops of the unnormalised kinds GK_HX1..GK_HW1: the
//                          tile is multiplied by 2^(-NH/2) after the last stage
//   PROG                   c128 offset of the op program in the item's matrices
//   G0                     program index of the pass's first op that reads its
//                          entry (a record or a matrix offset)
//   template <int S> static DOp stage(c128 (&a)[1 << R], DOp E, const DOp *prog, cmat *M)
//                          the ops of stage S in order (calls of jop and jopn
//                          below); E is the entry of the next op that reads
//                          one, the result likewise after the stage
#pragma once
#include "pass_kernels.h"

namespace vqc {

// op of kind KIND on register bits B0 (and B1) from its program entry E, or
// its adjoint (ADJ)
template <int R, bool ADJ, int KIND, int B0, int B1, int B2 = 0>
__device__ __forceinline__ void japply(c128 (&a)[1 << R], const DOp &E, cmat *mats) {
  constexpr int NR = 1 << R;
  SRec r;
  r.neg = E.neg;
  r.pad = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) r.ab[i] = E.ab[i];
  cmat *M = mats + E.g.mat;
  const uint32_t n = E.neg;
  if constexpr (KIND == GK_SXR1) {
    if (n & 1) rg_sxr1<NR, B0, ADJ, true>(a, r); else rg_sxr1<NR, B0, ADJ, false>(a, r);
  } else if constexpr (KIND == GK_SRR1) {
    if (n & 1) rg_srr1<NR, B0, ADJ, true>(a, r); else rg_srr1<NR, B0, ADJ, false>(a, r);
  } else if constexpr (KIND == GK_SPH1) {
    if (n & 1) rg_sph1<NR, B0, ADJ, true>(a, r); else rg_sph1<NR, B0, ADJ, false>(a, r);
  } else if constexpr (KIND == GK_SDG1) {
    switch (n & 3) {
      case 0: rg_sdg1<NR, B0, ADJ, false, false>(a, r); break;
      case 1: rg_sdg1<NR, B0, ADJ, true, false>(a, r); break;
      case 2: rg_sdg1<NR, B0, ADJ, false, true>(a, r); break;
      default: rg_sdg1<NR, B0, ADJ, true, true>(a, r); break;
    }
  } else if constexpr (KIND == GK_SRD1) {
    if (n & 2) rg_srd1<NR, B0, ADJ, true>(a, r); else rg_srd1<NR, B0, ADJ, false>(a, r);
  } else if constexpr (KIND == GK_SFX) {
    switch (n & 3) {
      case 0: rg_sfx<NR, B0, B1, ADJ, false, false>(a, r); break;
      case 1: rg_sfx<NR, B0, B1, ADJ, true, false>(a, r); break;
      case 2: rg_sfx<NR, B0, B1, ADJ, false, true>(a, r); break;
      default: rg_sfx<NR, B0, B1, ADJ, true, true>(a, r); break;
    }
  } else if constexpr (KIND == GK_HX1) {
    rg_hx1<NR, B0>(a);
  } else if constexpr (KIND == GK_HY1) {
    rg_hy1<NR, B0>(a);
  } else if constexpr (KIND == GK_HW1) {
    rg_hw1<NR, B0>(a);
  } else if constexpr (KIND == GK_DENSE1) {
    rg_dense1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_DIAG1) {
    rg_diag1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_XROT1) {
    rg_xrot1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_REAL1) {
    rg_real1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_RDIAG1) {
    rg_rdiag1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_PHASE1) {
    rg_phase1<NR, B0, ADJ>(a, M);
  } else if constexpr (KIND == GK_FSIMX) {
    rg_fsimx<NR, B0, B1, ADJ>(a, M);
  } else if constexpr (KIND == GK_DENSE2) {
    rg_dense2<NR, B0, B1, ADJ>(a, M);
  } else if constexpr (KIND == GK_DIAG2) {
    rg_diag2<NR, B0, B1, ADJ>(a, M);
  } else if constexpr (KIND == GK_FSIM) {
    rg_fsim<NR, B0, B1, ADJ>(a, M);
  } else if constexpr (KIND == GK_CX) {
    rg_cx<NR, B0, B1>(a);
  } else if constexpr (KIND == GK_DENSE3) {
    // bits fixed here: sorted bits and the index map are compile-time
    constexpr int lo = B0 < B1 ? (B0 < B2 ? B0 : B2) : (B1 < B2 ? B1 : B2);
    constexpr int hi = B0 > B1 ? (B0 > B2 ? B0 : B2) : (B1 > B2 ? B1 : B2);
    constexpr int mid = B0 + B1 + B2 - lo - hi;
    int rm[8];
    dense3_map(B0, B1, B2, rm);
    rg_dense3<NR, lo, mid, hi, ADJ>(a, M, rm);
  }
  // GK_NONE: nothing
}

// One op of the forward pass; E is its program entry, loaded by the previous
// op.  The entry at `next` is loaded here, after the wait for E and before
// E's arithmetic, so its scalar load overlaps this op.  The scheduling
// barriers keep the compiler from hoisting every op's load to the top of the
// pass (which would need far more scalar registers than there are) and from
// starting the next load before the wait (scalar loads return out of order,
// so a wait is a wait for all of them).
template <int R, int KIND, int B0, int B1, int B2 = 0>
__device__ __forceinline__ DOp jop(c128 (&a)[1 << R], const DOp &E, const DOp *next, cmat *mats) {
  lgkm_wait();
  const DOp En = ldc(next);
  __builtin_amdgcn_sched_barrier(0);
  japply<R, false, KIND, B0, B1, B2>(a, E, mats);
  __builtin_amdgcn_sched_barrier(0);
  return En;
}

// an op whose kind takes neither a record nor a matrix (controlled X, the
// unnormalised sqrt kinds): no program entry is read
template <int R, int KIND, int B0, int B1>
__device__ __forceinline__ void jopn(c128 (&a)[1 << R]) {
  constexpr int NR = 1 << R;
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (KIND == GK_CX) rg_cx<NR, B0, B1>(a);
  else if constexpr (KIND == GK_HX1) rg_hx1<NR, B0>(a);
  else if constexpr (KIND == GK_HY1) rg_hy1<NR, B0>(a);
  else if constexpr (KIND == GK_HW1) rg_hw1<NR, B0>(a);
  // GK_NONE: nothing
  __builtin_amdgcn_sched_barrier(0);
}

// LDS slot of tile-local index l under the pass's bank swizzle; linear over
// XOR, so the slot of base | o (disjoint bits) is jswz(base) ^ jswz(o) and a
// compile-time o costs one XOR
template <class P>
__device__ __forceinline__ int jswz(int l) {
  if constexpr (P::SWDEF) return l ^ (((l >> 4) ^ (l >> 8)) & 15);
  int n = 0;
#pragma unroll
  for (int q = 0; q < P::K; q++)
    if (P::SWC[q]) n ^= ((l >> q) & 1) ? P::SWC[q] : 0;
  return (l & ~((1 << P::SWB) - 1)) | n;
}

// tile-local index of lane t with zeros at stage S's register bits
template <class P, int S>
__device__ __forceinline__ int jbase(int t) {
  int base = t;
#pragma unroll
  for (int i = 0; i < P::R; i++) base = ins0<int>(base, P::SRT[S][i]);
  return base;
}

// tile-local offset of register j of stage S
template <class P, int S>
__device__ __forceinline__ constexpr int joff(int j) {
  int o = 0;
  for (int i = 0; i < P::R; i++)
    if ((j >> i) & 1) o |= 1 << P::RBIT[S][i];
  return o;
}

// Tile layouts over (lane t, register j): tile-local index lane(t) | reg(j).
// The load layout (registers over the top R tile bits, lanes over the rest),
// stage S's, and the store layout (lanes and registers in the order of the
// output's physical bits).  ROW: the layout's row in the pass's lane-slot
// table (the swizzled slot of lane(t), written by the planner).
template <class P>
struct JLoad {
  static constexpr int ROW = 0;
  __device__ static __forceinline__ int lane(int t) { return t; }
  __device__ static __forceinline__ constexpr int reg(int j) { return j << (P::K - P::R); }
};
template <class P, int S>
struct JStage {
  static constexpr int ROW = 1 + S;
  __device__ static __forceinline__ int lane(int t) { return jbase<P, S>(t); }
  __device__ static __forceinline__ constexpr int reg(int j) { return joff<P, S>(j); }
};
template <class P>
struct JStore {
  static constexpr int ROW = P::NST + 1;
  __device__ static __forceinline__ int lane(int t) {
    int sl = 0;
#pragma unroll
    for (int i = 0; i < P::K - P::R; i++)
      if ((t >> i) & 1) sl |= 1 << P::LBO[i];
    return sl;
  }
  __device__ static __forceinline__ constexpr int reg(int j) {
    int ol = 0;
    for (int i = 0; i < P::R; i++)
      if ((j >> i) & 1) ol |= 1 << P::LBO[P::K - P::R + i];
    return ol;
  }
};

template <bool SPLIT>
struct JLdsT {
  using T = c128;
};
template <>
struct JLdsT<true> {
  using T = double;
};

// a layout's slot of lane t as a byte offset into the LDS tile (tab: the
// pass's lane-slot table at lane t)
template <class P, class X>
__device__ __forceinline__ int jrow(const uint16_t *tab) {
  return tab[X::ROW << (P::K - P::R)];
}

// The registers of every lane from layout X (slot xs of lane t) to layout Y
// (slot ys) through the LDS tile.  SPLIT: the tile holds one double per
// amplitude and the real and imaginary halves go through it one after the
// other.  A lane's first write goes to the slots it read itself in the
// exchange before (X is that exchange's Y), so no barrier is needed before
// it.
template <class P, bool SPLIT, class X, class Y>
__device__ __forceinline__ void jxch(typename JLdsT<SPLIT>::T *buf, c128 (&a)[1 << P::R], int xs, int ys) {
  constexpr int NR = 1 << P::R;
  using T = typename JLdsT<SPLIT>::T;
  constexpr int W = sizeof(T);
  // xs, ys and the register offsets are byte offsets into the tile
  char *b = reinterpret_cast<char *>(buf);
  auto at = [&](int off) -> T & { return *reinterpret_cast<T *>(b + off); };
  if constexpr (!SPLIT) {
#pragma unroll
    for (int j = 0; j < NR; j++) at(xs ^ (jswz<P>(X::reg(j)) * W)) = a[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; j++) a[j] = at(ys ^ (jswz<P>(Y::reg(j)) * W));
  } else {
    double re[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) at(xs ^ (jswz<P>(X::reg(j)) * W)) = a[j].x;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; j++) re[j] = at(ys ^ (jswz<P>(Y::reg(j)) * W));
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; j++) at(xs ^ (jswz<P>(X::reg(j)) * W)) = a[j].y;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NR; j++) a[j] = make_double2(re[j], at(ys ^ (jswz<P>(Y::reg(j)) * W)));
  }
}

// the registers of the store layout to HBM (the pass's output layout)
template <class P>
__device__ __forceinline__ void jit_store_tile(const c128 (&a)[1 << P::R], gc128 *dst, int64_t tile, int t) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  uint64_t gbo = (uint64_t)tile;
#pragma unroll
  for (int i = 0; i < K; i++) gbo = ins0<uint64_t>(gbo, P::TQO[i]);
#pragma unroll
  for (int i = 0; i < K - R; i++)
    if ((t >> i) & 1) gbo |= 1ull << P::TQO[i];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    uint64_t oj = 0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if ((j >> i) & 1) oj |= 1ull << P::TQO[K - R + i];
    stg(&dst[gbo | oj], a[j]);
  }
}

// stages S .. NST-1 of one tile; a holds stage S's registers on entry
template <class P, bool SPLIT, int S>
__device__ __forceinline__ void jit_stages(typename JLdsT<SPLIT>::T *buf, c128 (&a)[1 << P::R], DOp E,
                                           const DOp *prog, cmat *MT, int t, uint64_t gbase, int64_t tile,
                                           gc128 *dst, const uint16_t *tab) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  // this exchange's slots, read before the stage's arithmetic hides them
  constexpr bool LAST = S == P::NST - 1;
  int xs = 0, ys = 0;
  if constexpr (!(LAST && P::DOUT)) {
    xs = jrow<P, JStage<P, S>>(tab);
    if constexpr (LAST) ys = jrow<P, JStore<P>>(tab);
    else ys = jrow<P, JStage<P, S + 1>>(tab);
  }
  E = P::template stage<S>(a, E, prog, MT);
  if constexpr (S == P::NST - 1) {
    if constexpr (P::NH > 0) {
      // the factor the unnormalised ops left out: 2^(-NH/2), a power of two
      // times 1/sqrt(2) for odd NH
      double f = (P::NH & 1) ? 0.70710678118654752440 : 1.0;
      for (int i = 0; i < P::NH / 2; i++) f *= 0.5;
#pragma unroll
      for (int j = 0; j < NR; j++) a[j] = make_double2(a[j].x * f, a[j].y * f);
    }
    if constexpr (P::DOUT) {
      // the last stage's wave lanes cover the low bits of the output layout:
      // store to HBM from registers (MOVES: local bit i at output bit TQL[i])
      const int base = jbase<P, S>(t);
      uint64_t gb = gbase;
      if constexpr (P::MOVES) {
        gb = (uint64_t)tile;
#pragma unroll
        for (int i = 0; i < K; i++) gb = ins0<uint64_t>(gb, P::TQO[i]);
      }
#pragma unroll
      for (int i = 0; i < K; i++)
        if ((base >> i) & 1) gb |= 1ull << (P::MOVES ? P::TQL[i] : P::TQ[i]);
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t go = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) go |= 1ull << (P::MOVES ? P::TQL[P::RBIT[S][i]] : P::TQ[P::RBIT[S][i]]);
        stg(&dst[gb | go], a[j]);
      }
    } else {
      jxch<P, SPLIT, JStage<P, S>, JStore<P>>(buf, a, xs, ys);
      jit_store_tile<P>(a, dst, tile, t);
    }
  } else {
    jxch<P, SPLIT, JStage<P, S>, JStage<P, S + 1>>(buf, a, xs, ys);
    jit_stages<P, SPLIT, S + 1>(buf, a, E, prog, MT, t, gbase, tile, dst, tab);
  }
}

// job of unit u: the only one, a division when every job has the same units,
// else a binary search over the job table
__device__ __forceinline__ int jit_job(const DJob *__restrict__ jobs, int n_jobs, int64_t u, const DOverride &ov) {
  if (n_jobs <= 1) return 0;
  if (ov.job_units > 0) return (int)(u / ov.job_units);
  return find_job(jobs, n_jobs, u);
}

// the 2^R amplitudes lane t holds of tile u (input layout), read from HBM.
// DIN: the registers are stage 0's and the lanes run over the other bits;
// else the load layout.  Either way the lanes run over the lowest tile bits
// first, so the loads are coalesced.
template <class P>
__device__ __forceinline__ void jit_load_tile(c128 (&r)[1 << P::R], const DJob *__restrict__ jobs, int n_jobs,
                                              int64_t u, const DOverride &ov, int t) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  const DJob J = ldc(&jobs[jit_job(jobs, n_jobs, u, ov)]);
  const gc128 *A = (const gc128 *)(ov.use ? ov.a : J.a);
  uint64_t g = (uint64_t)(u - J.unit0);
#pragma unroll
  for (int i = 0; i < K; i++) g = ins0<uint64_t>(g, P::TQ[i]);
  if constexpr (P::DIN) {
    const int base = jbase<P, 0>(t);
#pragma unroll
    for (int i = 0; i < K; i++)
      if ((base >> i) & 1) g |= 1ull << P::TQ[i];
  } else {
#pragma unroll
    for (int i = 0; i < K - R; i++) g |= (uint64_t)((t >> i) & 1) << P::TQ[i];
  }
#pragma unroll
  for (int j = 0; j < NR; j++) {
    uint64_t oj = 0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if ((j >> i) & 1) oj |= 1ull << P::TQ[P::DIN ? P::RBIT[0][i] : K - R + i];
    r[j] = ldg(&A[g | oj]);
  }
}

// One forward pass of pass description P over every tile of 2^K amplitudes
// of every job, 2^(K-R) threads per block.  PERSIST = false: one block per
// tile.  PERSIST = true: at most as many blocks as the chip holds at once,
// block b taking tiles b, b + grid, ..., each block reading its next tile
// from HBM into registers while the current tile's stages run.  SPLIT: the
// LDS tile holds doubles (see jxch).
template <class P, bool PERSIST, bool SPLIT>
__device__ __forceinline__ void jit_pass_fwd(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units,
                                             const DOverride &ov, const uint16_t *__restrict__ slots) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  __shared__ typename JLdsT<SPLIT>::T buf[1 << K];
  const int t = threadIdx.x;
  const uint16_t *tab = slots + P::TAB + t;
  int64_t u = blockIdx.x;
  if (u >= total_units) return;
  c128 pf[NR];
  jit_load_tile<P>(pf, jobs, n_jobs, u, ov, t);
  for (; u < total_units; u += PERSIST ? gridDim.x : total_units) {
    const DJob J = ldc(&jobs[jit_job(jobs, n_jobs, u, ov)]);
    const int64_t tile = u - J.unit0;
    gc128 *A = (gc128 *)(ov.use ? ov.a : J.a);
    gc128 *Bv = (gc128 *)(ov.use ? ov.b : J.b);
    cmat *MT = (cmat *)(ov.use ? ov.mats : J.mats);
    const DOp *prog = (const DOp *)(MT + P::PROG) + 1;
    const int mode = ov.use ? ov.mode : J.mode;
    gc128 *dst = mode == 1 ? Bv : A;
    uint64_t gbase = (uint64_t)tile;
#pragma unroll
    for (int i = 0; i < K; i++) gbase = ins0<uint64_t>(gbase, P::TQ[i]);
    c128 a[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) a[j] = pf[j];
    if constexpr (PERSIST) {
      const int64_t un = u + gridDim.x;
      if (un < total_units) jit_load_tile<P>(pf, jobs, n_jobs, un, ov, t);
    }
    if constexpr (P::NST == 0) {
      // a pass without ops only moves qubits
      jxch<P, SPLIT, JLoad<P>, JStore<P>>(buf, a, jrow<P, JLoad<P>>(tab), jrow<P, JStore<P>>(tab));
      jit_store_tile<P>(a, dst, tile, t);
    } else {
      if constexpr (!P::DIN) jxch<P, SPLIT, JLoad<P>, JStage<P, 0>>(buf, a, jrow<P, JLoad<P>>(tab), jrow<P, JStage<P, 0>>(tab));
      jit_stages<P, SPLIT, 0>(buf, a, ldc(prog + P::G0), prog, MT, t, gbase, tile, dst, tab);
    }
    __syncthreads();  // the next tile overwrites the LDS tile
  }
}

// ------------------------------------------------------------ adjoint pass
// Alg. 2 for one pass, as k_pass_lds<K,R,1> does it: the pass's ops in
// reverse, Phi <- Q^dagger Phi and Psi <- Q^dagger Psi, and for every
// parameter of an op the partial inner product Re<Psi| dQ |Phi> of the tile,
// summed over a wave and written to the pass's reduction slot.  The pass
// description P adds
//   NVAR, VSLOT[NVAR]      the pass's derivative slots and their rows in the
//                          partials array
//   DIN                    the first stage (in reverse order) holds none of the
//                          low bits: it reads HBM directly (DOUT likewise for
//                          the last one)
//   template <int S> static DOp astage(a, b, E, prog, M, red, lane, wave)
//                          stage S's ops in reverse (calls of the helpers below)

// wave sum of a tile's partial, stored by the wave's last lane (which holds
// it) into the reduction slot
template <int WS, int NW>
__device__ __forceinline__ void jred(double (*red)[NW], int slot, double v, int lane, int wave) {
  v = wave_sum_last<WS>(v);
  if (lane == WS - 1) red[slot][wave] = v;
}

// Re<b| D |a> over the lane's groups for a derivative matrix D of kind DK
template <int R, int DK, int B0, int B1>
__device__ __forceinline__ double jgrad(const c128 (&a)[1 << R], const c128 (&b)[1 << R], cmat *D) {
  constexpr int NR = 1 << R;
  if constexpr (DK == GK_DENSE1) return gr_dense1<NR, B0>(a, b, D);
  else if constexpr (DK == GK_DIAG1) return gr_diag1<NR, B0>(a, b, D);
  else if constexpr (DK == GK_DENSE2) return gr_dense2<NR, B0, B1>(a, b, D);
  else if constexpr (DK == GK_GENX || DK == GK_GENY || DK == GK_GENZ) return gr_gen<NR, B0, DK>(a, b);
  else return 0.0;
}

// LDS slot of register j of stage S for lane base `base`
template <class P, int S>
__device__ __forceinline__ int jslot(int base, int j) {
  return jswz<P>(base) ^ jswz<P>(joff<P, S>(j));
}

// a tile (in LDS) to HBM in the pass's output layout
template <class P>
__device__ __forceinline__ void jit_store_out(const c128 *lx, gc128 *dst, int64_t tile, int t) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  uint64_t gbo = (uint64_t)tile;
#pragma unroll
  for (int i = 0; i < K; i++) gbo = ins0<uint64_t>(gbo, P::TQO[i]);
  uint64_t so = 0;
  int sl = 0;
#pragma unroll
  for (int i = 0; i < K - R; i++)
    if ((t >> i) & 1) {
      so |= 1ull << P::TQO[i];
      sl |= 1 << P::LBO[i];
    }
#pragma unroll
  for (int j = 0; j < NR; j++) {
    uint64_t oj = 0;
    int ol = 0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if ((j >> i) & 1) {
        oj |= 1ull << P::TQO[K - R + i];
        ol |= 1 << P::LBO[K - R + i];
      }
    stg(&dst[gbo | so | oj], lx[jswz<P>(sl) ^ jswz<P>(ol)]);
  }
}

// a tile from HBM (input layout, lanes over the low tile bits) into LDS
template <class P>
__device__ __forceinline__ void jit_load_in(c128 *lx, const gc128 *src, uint64_t gbase, int t) {
  constexpr int K = P::K, R = P::R, NR = 1 << R, T = 1 << (K - R);
  uint64_t st = 0;
#pragma unroll
  for (int i = 0; i < K - R; i++) st |= (uint64_t)((t >> i) & 1) << P::TQ[i];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    uint64_t oj = 0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if ((j >> i) & 1) oj |= 1ull << P::TQ[K - R + i];
    lx[jswz<P>(t) ^ jswz<P>(j * T)] = ldg(&src[gbase | st | oj]);
  }
}

// Stages S .. 0 (reverse order) of one tile; a and b hold stage S's registers
// on entry.  SH: Phi and Psi share one LDS tile, exchanged one after the
// other (half the LDS of two tiles, so twice the resident blocks, for two
// more barriers per stage change).
template <class P, int S, int NW, bool SH>
__device__ __forceinline__ void jit_astages(c128 *la, c128 *lb, c128 (&a)[1 << P::R], c128 (&b)[1 << P::R], DOp E,
                                            const DOp *prog, cmat *MT, int t, uint64_t gbase, int64_t tile,
                                            gc128 *dst, gc128 *dstb, double (*red)[NW]) {
  if constexpr (S >= 0) {
    constexpr int K = P::K, R = P::R, NR = 1 << R;
    const int lane = t & 63, wave = t >> 6;
    const int base = jbase<P, S>(t);
    E = P::template astage<S>(a, b, E, prog, MT, red, lane, wave);
    if constexpr (S == 0 && P::DOUT) {
      uint64_t gb = gbase;
#pragma unroll
      for (int i = 0; i < K; i++)
        if ((base >> i) & 1) gb |= 1ull << P::TQ[i];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t go = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) go |= 1ull << P::TQ[P::RBIT[S][i]];
        stg(&dst[gb | go], a[j]);
        stg(&dstb[gb | go], b[j]);
      }
      __syncthreads();  // every wave's reduction entries are written
    } else if constexpr (S == 0) {
#pragma unroll
      for (int j = 0; j < NR; j++) la[jslot<P, S>(base, j)] = a[j];
      if constexpr (!SH)
#pragma unroll
        for (int j = 0; j < NR; j++) lb[jslot<P, S>(base, j)] = b[j];
      __syncthreads();
      jit_store_out<P>(la, dst, tile, t);
      if constexpr (SH) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; j++) la[jslot<P, S>(base, j)] = b[j];
        __syncthreads();
        jit_store_out<P>(la, dstb, tile, t);
      } else {
        jit_store_out<P>(lb, dstb, tile, t);
      }
    } else {
      const int nb = jbase<P, S - 1>(t);
#pragma unroll
      for (int j = 0; j < NR; j++) la[jslot<P, S>(base, j)] = a[j];
      if constexpr (!SH)
#pragma unroll
        for (int j = 0; j < NR; j++) lb[jslot<P, S>(base, j)] = b[j];
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NR; j++) a[j] = la[jslot<P, S - 1>(nb, j)];
      if constexpr (SH) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; j++) la[jslot<P, S>(base, j)] = b[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; j++) b[j] = la[jslot<P, S - 1>(nb, j)];
      } else {
#pragma unroll
        for (int j = 0; j < NR; j++) b[j] = lb[jslot<P, S - 1>(nb, j)];
      }
      // (the next write to LDS, after the next stage's ops, goes to the slots
      // each lane has just read itself: no barrier needed before it)
      jit_astages<P, S - 1, NW, SH>(la, lb, a, b, E, prog, MT, t, gbase, tile, dst, dstb, red);
    }
  }
}

// One adjoint pass of description P: a block per tile, the per-tile partial
// of each derivative slot written to the item's partials array (summed over
// tiles afterwards in a fixed order).
template <class P, bool SH>
__device__ __forceinline__ void jit_pass_adj(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units,
                                             const DOverride &ov) {
  constexpr int K = P::K, R = P::R, NR = 1 << R, T = 1 << (K - R);
  constexpr int NW = (T + 63) / 64;
  __shared__ c128 la[1 << K];
  __shared__ c128 lb[SH ? 1 : (1 << K)];
  __shared__ double red[P::NVAR > 0 ? P::NVAR : 1][NW];
  const int t = threadIdx.x;
  const int64_t u = blockIdx.x;
  if (u >= total_units) return;
  const DJob J = ldc(&jobs[jit_job(jobs, n_jobs, u, ov)]);
  const int64_t tile = u - J.unit0;
  const gc128 *src = (const gc128 *)(ov.use ? ov.a : J.a);
  const gc128 *srcb = (const gc128 *)(ov.use ? ov.b : J.b);
  gc128 *dst = (gc128 *)(ov.use ? ov.a : J.a);
  gc128 *dstb = (gc128 *)(ov.use ? ov.b : J.b);
  if ((ov.use ? ov.mode : J.mode) == 1) {
    dst = (gc128 *)(ov.use ? ov.a2 : J.a2);
    dstb = (gc128 *)(ov.use ? ov.b2 : J.b2);
  }
  cmat *MT = (cmat *)(ov.use ? ov.mats : J.mats);
  const DOp *prog = (const DOp *)(MT + P::PROG) + 1;
  double *PT = ov.use ? ov.partials : J.partials;
  uint64_t gbase = (uint64_t)tile;
#pragma unroll
  for (int i = 0; i < K; i++) gbase = ins0<uint64_t>(gbase, P::TQ[i]);
  const DOp E = ldc(prog + P::GLAST);  // the pass's last op runs first
  if constexpr (P::NST == 0) {
    // a pass without ops only moves qubits
    jit_load_in<P>(la, src, gbase, t);
    __syncthreads();
    jit_store_out<P>(la, dst, tile, t);
    __syncthreads();
    jit_load_in<P>(la, srcb, gbase, t);
    __syncthreads();
    jit_store_out<P>(la, dstb, tile, t);
  } else {
    constexpr int S = P::NST - 1;
    c128 a[NR], b[NR];
    const int base = jbase<P, S>(t);
    if constexpr (P::DIN) {
      // the first stage's lanes run over the low tile bits: read HBM directly
      uint64_t gb = gbase;
#pragma unroll
      for (int i = 0; i < K; i++)
        if ((base >> i) & 1) gb |= 1ull << P::TQ[i];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t go = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) go |= 1ull << P::TQ[P::RBIT[S][i]];
        a[j] = ldg(&src[gb | go]);
        b[j] = ldg(&srcb[gb | go]);
      }
    } else {
      jit_load_in<P>(la, src, gbase, t);
      if constexpr (!SH) jit_load_in<P>(lb, srcb, gbase, t);
      __syncthreads();
#pragma unroll
      for (int j = 0; j < NR; j++) a[j] = la[jslot<P, S>(base, j)];
      if constexpr (SH) {
        __syncthreads();
        jit_load_in<P>(la, srcb, gbase, t);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; j++) b[j] = la[jslot<P, S>(base, j)];
      } else {
#pragma unroll
        for (int j = 0; j < NR; j++) b[j] = lb[jslot<P, S>(base, j)];
      }
    }
    jit_astages<P, S, NW, SH>(la, lb, a, b, E, prog, MT, t, gbase, tile, dst, dstb, red);
  }
  if constexpr (P::NVAR > 0) {
    for (int v = t; v < P::NVAR; v += T) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; w++) sum += red[v][w];
      PT[(int64_t)P::VSLOT[v] * J.n_units + tile] = sum;
    }
  }
}

// ---------------------------------------------- adjoint pass on lane slots
// The same step of Alg. 2 with the forward pass's tile machinery: the tile's
// layouts exchanged through LDS by jxch (SPLIT: as real and imaginary halves,
// half the LDS), lane slots read from the planner's table (P::TAB), Phi and
// Psi moved one after the other through the one tile.

// the 2^R amplitudes of lane t in the load layout, read from HBM
template <class P>
__device__ __forceinline__ void jit_load_regs(c128 (&r)[1 << P::R], const gc128 *src, uint64_t gbase, int t) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  uint64_t g = gbase;
#pragma unroll
  for (int i = 0; i < K - R; i++) g |= (uint64_t)((t >> i) & 1) << P::TQ[i];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    uint64_t oj = 0;
#pragma unroll
    for (int i = 0; i < R; i++)
      if ((j >> i) & 1) oj |= 1ull << P::TQ[K - R + i];
    r[j] = ldg(&src[g | oj]);
  }
}

// stages S .. 0 (reverse order); a and b hold stage S's registers on entry
template <class P, bool SPLIT, int S, int NW>
__device__ __forceinline__ void jit_astages2(typename JLdsT<SPLIT>::T *buf, c128 (&a)[1 << P::R],
                                             c128 (&b)[1 << P::R], DOp E, const DOp *prog, cmat *MT, int t,
                                             uint64_t gbase, int64_t tile, gc128 *dst, gc128 *dstb,
                                             double (*red)[NW], const uint16_t *tab) {
  constexpr int K = P::K, R = P::R, NR = 1 << R;
  const int lane = t & 63, wave = t >> 6;
  // this stage's exchange slots, read before its arithmetic hides them
  int xs = 0, ys = 0;
  if constexpr (!(S == 0 && P::DOUT)) {
    xs = jrow<P, JStage<P, S>>(tab);
    if constexpr (S == 0) ys = jrow<P, JStore<P>>(tab);
    else ys = jrow<P, JStage<P, (S > 0 ? S - 1 : 0)>>(tab);
  }
  E = P::template astage<S>(a, b, E, prog, MT, red, lane, wave);
  if constexpr (S == 0) {
    if constexpr (P::DOUT) {
      const int base = jbase<P, 0>(t);
      uint64_t gb = gbase;
#pragma unroll
      for (int i = 0; i < K; i++)
        if ((base >> i) & 1) gb |= 1ull << P::TQ[i];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t go = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) go |= 1ull << P::TQ[P::RBIT[0][i]];
        stg(&dst[gb | go], a[j]);
        stg(&dstb[gb | go], b[j]);
      }
      __syncthreads();  // every wave's reduction entries are written
    } else {
      jxch<P, SPLIT, JStage<P, 0>, JStore<P>>(buf, a, xs, ys);
      jit_store_tile<P>(a, dst, tile, t);
      __syncthreads();  // other lanes may still read Phi from this lane's stage slots
      jxch<P, SPLIT, JStage<P, 0>, JStore<P>>(buf, b, xs, ys);
      jit_store_tile<P>(b, dstb, tile, t);
    }
  } else {
    jxch<P, SPLIT, JStage<P, S>, JStage<P, S - 1>>(buf, a, xs, ys);
    __syncthreads();
    jxch<P, SPLIT, JStage<P, S>, JStage<P, S - 1>>(buf, b, xs, ys);
    jit_astages2<P, SPLIT, S - 1, NW>(buf, a, b, E, prog, MT, t, gbase, tile, dst, dstb, red, tab);
  }
}

template <class P, bool SPLIT>
__device__ __forceinline__ void jit_pass_adj2(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units,
                                              const DOverride &ov, const uint16_t *__restrict__ slots) {
  constexpr int K = P::K, R = P::R, NR = 1 << R, T = 1 << (K - R);
  constexpr int NW = (T + 63) / 64;
  __shared__ typename JLdsT<SPLIT>::T buf[1 << K];
  __shared__ double red[P::NVAR > 0 ? P::NVAR : 1][NW];
  const int t = threadIdx.x;
  const int64_t u = blockIdx.x;
  if (u >= total_units) return;
  const uint16_t *tab = slots + P::TAB + t;
  const DJob J = ldc(&jobs[jit_job(jobs, n_jobs, u, ov)]);
  const int64_t tile = u - J.unit0;
  const gc128 *src = (const gc128 *)(ov.use ? ov.a : J.a);
  const gc128 *srcb = (const gc128 *)(ov.use ? ov.b : J.b);
  gc128 *dst = (gc128 *)(ov.use ? ov.a : J.a);
  gc128 *dstb = (gc128 *)(ov.use ? ov.b : J.b);
  if ((ov.use ? ov.mode : J.mode) == 1) {
    dst = (gc128 *)(ov.use ? ov.a2 : J.a2);
    dstb = (gc128 *)(ov.use ? ov.b2 : J.b2);
  }
  cmat *MT = (cmat *)(ov.use ? ov.mats : J.mats);
  const DOp *prog = (const DOp *)(MT + P::PROG) + 1;
  double *PT = ov.use ? ov.partials : J.partials;
  uint64_t gbase = (uint64_t)tile;
#pragma unroll
  for (int i = 0; i < K; i++) gbase = ins0<uint64_t>(gbase, P::TQ[i]);
  c128 a[NR], b[NR];
  if constexpr (P::NST == 0) {
    // a pass without ops only moves qubits
    const int xs = jrow<P, JLoad<P>>(tab), ys = jrow<P, JStore<P>>(tab);
    jit_load_regs<P>(a, src, gbase, t);
    jxch<P, SPLIT, JLoad<P>, JStore<P>>(buf, a, xs, ys);
    jit_store_tile<P>(a, dst, tile, t);
    jit_load_regs<P>(b, srcb, gbase, t);
    __syncthreads();
    jxch<P, SPLIT, JLoad<P>, JStore<P>>(buf, b, xs, ys);
    jit_store_tile<P>(b, dstb, tile, t);
  } else {
    constexpr int S = P::NST - 1;
    const DOp E = ldc(prog + P::GLAST);  // the pass's last op runs first
    if constexpr (P::DIN) {
      // the first stage's lanes run over the low tile bits: read HBM directly
      const int base = jbase<P, S>(t);
      uint64_t gb = gbase;
#pragma unroll
      for (int i = 0; i < K; i++)
        if ((base >> i) & 1) gb |= 1ull << P::TQ[i];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t go = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) go |= 1ull << P::TQ[P::RBIT[S][i]];
        a[j] = ldg(&src[gb | go]);
        b[j] = ldg(&srcb[gb | go]);
      }
    } else {
      const int xs = jrow<P, JLoad<P>>(tab), ys = jrow<P, JStage<P, S>>(tab);
      jit_load_regs<P>(a, src, gbase, t);
      jit_load_regs<P>(b, srcb, gbase, t);
      jxch<P, SPLIT, JLoad<P>, JStage<P, S>>(buf, a, xs, ys);
      __syncthreads();
      jxch<P, SPLIT, JLoad<P>, JStage<P, S>>(buf, b, xs, ys);
    }
    jit_astages2<P, SPLIT, S, NW>(buf, a, b, E, prog, MT, t, gbase, tile, dst, dstb, red, tab);
  }
  if constexpr (P::NVAR > 0) {
    for (int v = t; v < P::NVAR; v += T) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; w++) sum += red[v][w];
      PT[(int64_t)P::VSLOT[v] * J.n_units + tile] = sum;
    }
  }
}

}  // namespace vqc

// gfx950 (CDNA4) kernels of the variational-circuit hot path.
//
// All amplitudes are complex128 (double2), 16 B.  The state is HBM-resident;
// every kernel here is a streaming pass whose roofline is HBM bandwidth (a
// 1q gate is 14 flop per 32 B moved), so the design goal is few passes with
// fully used 128 B lines, not MFMA: the only dense contraction is a 2^m x 2^m
// matrix times many short vectors, m <= 4.
//
//   k_pass_lds   fused pass (Sec. 3.2's aggregation idea taken to a tile):
//                a tile of 2^K amplitudes -- the low c qubits, contiguous in
//                memory, plus K-c chosen higher qubits -- is staged in LDS; a
//                run of ops on the tile's qubits is applied in register
//                "stages" of 2^R amplitudes per lane; one HBM read and one
//                write per pass.  ADJ=true is the fused adjoint step of
//                Alg. 2 on Phi and Psi together, with per-op FP64 partial
//                inner products reduced deterministically.
//   k_pass_reg   register-only pass (tile = the 2^R amplitudes of one lane);
//                used for vec(rho) superoperators and small states.  MODE 2
//                is the noisy adjoint step of Sec. 3.5 with Phi recomputed
//                from the pass-start checkpoint.
//   k_g*         single-op kernels (Eq. (3), Eq. (twoqubitgate), and the
//                structured gates of Sec. 2.2 that touch only the amplitudes
//                that change).
//   k_expect     Pauli-sum expectation / adjoint seed H psi (Sec. 2.5,
//                Alg. 2 initialisation) with a two-stage deterministic sum.
#pragma once
#include "vqc_internal.h"
#include "../../include/vqc.h"

namespace vqc {

// --------------------------------------------------------- address spaces
// Descriptors and gate matrices are written before a pass kernel starts and
// only read during it: reading them through the constant address space lets
// the compiler use scalar (uniform) loads instead of per-lane loads that
// serialise on memory latency.  The state goes through the global address
// space (global_load/store rather than flat, which would also hold LDS waits).
#define VQC_AS_CONST __attribute__((address_space(4)))
#define VQC_AS_GLOBAL __attribute__((address_space(1)))
typedef double v2d __attribute__((ext_vector_type(2)));
typedef const VQC_AS_CONST v2d cmat;  // matrix element, scalar-loaded
typedef VQC_AS_GLOBAL v2d gc128;      // state amplitude in HBM

// whole-dword scalar loads (scalar loads have no byte/short forms); the
// fields are then extracted in registers
template <typename T>
__device__ __forceinline__ T ldc(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size must be a multiple of 4 bytes");
  constexpr int W = sizeof(T) / 4;
  union {
    T t;
    uint32_t w[W];
  } u;
  const VQC_AS_CONST uint32_t *q = (const VQC_AS_CONST uint32_t *)p;
#pragma unroll
  for (int i = 0; i < W; i++) u.w[i] = q[i];
  return u.t;
}

// ------------------------------------------------------------ complex math

__device__ __forceinline__ c128 cmul(c128 a, c128 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a*b + c
__device__ __forceinline__ c128 cfma(c128 a, c128 b, c128 c) {
  return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ c128 cconj(c128 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ c128 cadd(c128 a, c128 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c128 cscale(double s, c128 a) { return make_double2(s * a.x, s * a.y); }
// Re(conj(a) * b)
__device__ __forceinline__ double redot(c128 a, c128 b) { return fma(a.x, b.x, a.y * b.y); }

__device__ __forceinline__ c128 tc(v2d v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ v2d tv(c128 c) {
  v2d v;
  v.x = c.x;
  v.y = c.y;
  return v;
}

// streaming state access: every amplitude is read and written once per
// pass, so loads and stores carry the nontemporal hint
__device__ __forceinline__ c128 ldg(const gc128 *p) { return tc(__builtin_nontemporal_load(p)); }
__device__ __forceinline__ void stg(gc128 *p, c128 v) { __builtin_nontemporal_store(tv(v), p); }

// element (r, c) of M (row-major D x D) or of M^dagger
template <bool ADJ, int D>
__device__ __forceinline__ c128 mel(cmat *M, int r, int c) {
  if (ADJ) return cconj(tc(M[c * D + r]));
  return tc(M[r * D + c]);
}

// insert a zero bit at position p
template <typename U>
__device__ __forceinline__ U ins0(U x, int p) {
  const U low = x & ((U(1) << p) - 1);
  return ((x >> p) << (p + 1)) | low;
}

// LDS index swizzle: xor bits 4..11 into bits 0..3 (bijective, keeps each
// 16-element group inside itself) so that register stages whose lanes stride
// by 2^k elements spread over banks.
__device__ __forceinline__ int swz(int l) { return l ^ (((l >> 4) ^ (l >> 8)) & 15); }

// ------------------------------------------------- register-level op kernels

template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_dense1(c128 (&a)[NR], cmat *M) {
  const c128 m00 = mel<ADJ, 2>(M, 0, 0), m01 = mel<ADJ, 2>(M, 0, 1);
  const c128 m10 = mel<ADJ, 2>(M, 1, 0), m11 = mel<ADJ, 2>(M, 1, 1);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = cfma(m00, x, cmul(m01, y));
    a[k] = cfma(m10, x, cmul(m11, y));
  }
}

template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_diag1(c128 (&a)[NR], cmat *M) {
  const c128 d0 = mel<ADJ, 2>(M, 0, 0), d1 = mel<ADJ, 2>(M, 1, 1);
#pragma unroll
  for (int j = 0; j < NR; j++) a[j] = cmul((j >> B) & 1 ? d1 : d0, a[j]);
}

// [[a, i b], [i c, d]] with real a, b, c, d: 4 FP64 ops per output
template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_xrot1(c128 (&a)[NR], cmat *M) {
  const double m00 = M[0].x, m11 = M[3].x;
  // adjoint: [[a, -i c], [-i b, d]]
  const double b = ADJ ? -M[2].y : M[1].y, c = ADJ ? -M[1].y : M[2].y;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(fma(m00, x.x, -b * y.y), fma(m00, x.y, b * y.x));
    a[k] = make_double2(fma(m11, y.x, -c * x.y), fma(m11, y.y, c * x.x));
  }
}

// real 2x2: 4 FP64 ops per output
template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_real1(c128 (&a)[NR], cmat *M) {
  const double m00 = M[0].x, m11 = M[3].x;
  const double m01 = ADJ ? M[2].x : M[1].x, m10 = ADJ ? M[1].x : M[2].x;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(fma(m00, x.x, m01 * y.x), fma(m00, x.y, m01 * y.y));
    a[k] = make_double2(fma(m10, x.x, m11 * y.x), fma(m10, x.y, m11 * y.y));
  }
}

// real diagonal, complex off-diagonal: 6 FP64 ops per output
template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_rdiag1(c128 (&a)[NR], cmat *M) {
  const double m00 = M[0].x, m11 = M[3].x;
  const c128 m01 = ADJ ? cconj(tc(M[2])) : tc(M[1]), m10 = ADJ ? cconj(tc(M[1])) : tc(M[2]);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(fma(m00, x.x, fma(m01.x, y.x, -m01.y * y.y)), fma(m00, x.y, fma(m01.x, y.y, m01.y * y.x)));
    a[k] = make_double2(fma(m11, y.x, fma(m10.x, x.x, -m10.y * x.y)), fma(m11, y.y, fma(m10.x, x.y, m10.y * x.x)));
  }
}

// diag(1, m11): only the |1> half changes
template <int NR, int B, bool ADJ>
__device__ __forceinline__ void rg_phase1(c128 (&a)[NR], cmat *M) {
  const c128 d1 = mel<ADJ, 2>(M, 1, 1);
#pragma unroll
  for (int j = 0; j < NR; j++)
    if ((j >> B) & 1) a[j] = cmul(d1, a[j]);
}

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_dense2(c128 (&a)[NR], cmat *M) {
  c128 m[16];
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int c = 0; c < 4; c++) m[r * 4 + c] = mel<ADJ, 4>(M, r, c);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    int idx[4];
#pragma unroll
    for (int l = 0; l < 4; l++) idx[l] = j | ((l & 1) << B0) | ((l >> 1) << B1);
    c128 x[4];
#pragma unroll
    for (int l = 0; l < 4; l++) x[l] = a[idx[l]];
#pragma unroll
    for (int r = 0; r < 4; r++) {
      c128 acc = cmul(m[r * 4 + 0], x[0]);
      acc = cfma(m[r * 4 + 1], x[1], acc);
      acc = cfma(m[r * 4 + 2], x[2], acc);
      acc = cfma(m[r * 4 + 3], x[3], acc);
      a[idx[r]] = acc;
    }
  }
}

// 8x8 on register bits S0, S1, S2; the matrix element for the group's local
// indices (r, c) (l = b_{S0} + 2 b_{S1} + 4 b_{S2}) is M[rm[r]][rm[c]] (or
// its adjoint's), rm mapping these local indices to the op's own (which
// orders its qubits differently when rm is not the identity)
template <int NR, int S0, int S1, int S2, bool ADJ>
__device__ __forceinline__ void rg_dense3(c128 (&a)[NR], cmat *M, const int (&rm)[8]) {
  if constexpr (NR >= 8) {
#pragma unroll
    for (int j = 0; j < NR; j++) {
      if (j & ((1 << S0) | (1 << S1) | (1 << S2))) continue;
      int idx[8];
#pragma unroll
      for (int l = 0; l < 8; l++) idx[l] = j | ((l & 1) << S0) | (((l >> 1) & 1) << S1) | ((l >> 2) << S2);
      c128 x[8];
#pragma unroll
      for (int l = 0; l < 8; l++) x[l] = a[idx[l]];
#pragma unroll
      for (int r = 0; r < 8; r++) {
        c128 acc = cmul(mel<ADJ, 8>(M, rm[r], rm[0]), x[0]);
#pragma unroll
        for (int c = 1; c < 8; c++) acc = cfma(mel<ADJ, 8>(M, rm[r], rm[c]), x[c], acc);
        a[idx[r]] = acc;
      }
    }
  }
}

// the op's register bits (any order, distinct) as sorted bits and the local
// index map of rg_dense3
__device__ __forceinline__ int dense3_map(int r0, int r1, int r2, int (&rm)[8]) {
  const int lo = min(r0, min(r1, r2)), hi = max(r0, max(r1, r2)), mid = r0 + r1 + r2 - lo - hi;
  const int pos[3] = {r0 == lo ? 0 : r0 == mid ? 1 : 2, r1 == lo ? 0 : r1 == mid ? 1 : 2,
                      r2 == lo ? 0 : r2 == mid ? 1 : 2};
#pragma unroll
  for (int l = 0; l < 8; l++) {
    int o = 0;
#pragma unroll
    for (int t = 0; t < 3; t++) o |= ((l >> pos[t]) & 1) << t;
    rm[l] = o;
  }
  return (1 << lo) | (1 << mid) | (1 << hi);
}

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_diag2(c128 (&a)[NR], cmat *M) {
  c128 d[4];
#pragma unroll
  for (int l = 0; l < 4; l++) d[l] = mel<ADJ, 4>(M, l, l);
#pragma unroll
  for (int j = 0; j < NR; j++) a[j] = cmul(d[((j >> B0) & 1) | (((j >> B1) & 1) << 1)], a[j]);
}

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_fsim(c128 (&a)[NR], cmat *M) {
  const c128 m00 = mel<ADJ, 4>(M, 0, 0), m11 = mel<ADJ, 4>(M, 1, 1), m12 = mel<ADJ, 4>(M, 1, 2);
  const c128 m21 = mel<ADJ, 4>(M, 2, 1), m22 = mel<ADJ, 4>(M, 2, 2), m33 = mel<ADJ, 4>(M, 3, 3);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    const int i1 = j | (1 << B0), i2 = j | (1 << B1), i3 = i1 | i2;
    const c128 x1 = a[i1], x2 = a[i2];
    a[j] = cmul(m00, a[j]);
    a[i1] = cfma(m11, x1, cmul(m12, x2));
    a[i2] = cfma(m21, x1, cmul(m22, x2));
    a[i3] = cmul(m33, a[i3]);
  }
}

// fSim with Delta = 0: |00> unchanged, XROT block on |01>,|10>, phase on |11>
template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_fsimx(c128 (&a)[NR], cmat *M) {
  const double c1 = M[5].x, c2 = M[10].x;
  const double s12 = ADJ ? -M[9].y : M[6].y, s21 = ADJ ? -M[6].y : M[9].y;
  const c128 m33 = mel<ADJ, 4>(M, 3, 3);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    const int i1 = j | (1 << B0), i2 = j | (1 << B1), i3 = i1 | i2;
    const c128 x = a[i1], y = a[i2];
    a[i1] = make_double2(fma(c1, x.x, -s12 * y.y), fma(c1, x.y, s12 * y.x));
    a[i2] = make_double2(fma(c2, y.x, -s21 * x.y), fma(c2, y.y, s21 * x.x));
    a[i3] = cmul(m33, a[i3]);
  }
}

template <int NR, int B0, int B1>
__device__ __forceinline__ void rg_cx(c128 (&a)[NR]) {
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (!((j >> B0) & 1) || ((j >> B1) & 1)) continue;
    const int k = j | (1 << B1);
    const c128 t = a[j];
    a[j] = a[k];
    a[k] = t;
  }
}

// a I + b |I>><<I| on four bits (ket pair, bra pair): every entry scaled by
// a, and b times the sum of the four diagonal entries (x = y: local 0, 5,
// 10, 15) added to each of them; real and symmetric, so its adjoint is itself
template <int NR>
__device__ __forceinline__ void rg_depol4(c128 (&a)[NR], cmat *M) {
  if constexpr (NR == 16) {
    const double al = M[1 * 16 + 1].x, be = M[0 * 16 + 5].x;
    const double sr = (a[0].x + a[5].x) + (a[10].x + a[15].x);
    const double si = (a[0].y + a[5].y) + (a[10].y + a[15].y);
#pragma unroll
    for (int l = 0; l < 16; l++) {
      a[l].x *= al;
      a[l].y *= al;
    }
#pragma unroll
    for (int l = 0; l < 16; l += 5) {
      a[l].x = fma(be, sr, a[l].x);
      a[l].y = fma(be, si, a[l].y);
    }
  }
}

template <int NR, bool ADJ>
__device__ __forceinline__ void rg_dense4(c128 (&a)[NR], cmat *M) {
  if constexpr (NR == 16) {
    c128 x[16];
#pragma unroll
    for (int l = 0; l < 16; l++) x[l] = a[l];
#pragma unroll
    for (int r = 0; r < 16; r++) {
      c128 acc = cmul(mel<ADJ, 16>(M, r, 0), x[0]);
#pragma unroll
      for (int c = 1; c < 16; c++) acc = cfma(mel<ADJ, 16>(M, r, c), x[c], acc);
      a[r] = acc;
    }
  }
}

// ------------------------------------------- in-place rotation (shear) forms
// A plane rotation [[C, -S], [S, C]] of (u, v) is three shears
// u += a v; v += b u; u += a v with a = -tan(p/2) = -S/(1+C), b = S, each a
// fused multiply-add accumulated into the coordinate's own register, so a
// run of these ops keeps every amplitude in place (no register copies
// between ops) and costs 3 FP64 FMAs per rotated pair of reals instead of 4.
// The record keeps C >= 0 (|a| <= 1, no cancellation); a rotation with
// C < 0 is stored as the rotation by p - pi followed by a negation, folded
// into the last two FMAs.
template <bool NEG>
__device__ __forceinline__ void shr(double &u, double &v, double a, double b) {
  u = fma(a, v, u);
  if (!NEG) {
    v = fma(b, u, v);
    u = fma(a, v, u);
  } else {
    v = fma(-b, u, -v);
    u = fma(a, v, -u);
  }
}

// sqrt(2) sqrt(X) (phase-factored): x' = x - i y, y' = y - i x
template <int NR, int B>
__device__ __forceinline__ void rg_hx1(c128 (&a)[NR]) {
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(x.x + y.y, x.y - y.x);
    a[k] = make_double2(y.x + x.y, y.y - x.x);
  }
}

// sqrt(2) sqrt(Y) (phase-factored): x' = x - y, y' = x + y
template <int NR, int B>
__device__ __forceinline__ void rg_hy1(c128 (&a)[NR]) {
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(x.x - y.x, x.y - y.y);
    a[k] = make_double2(x.x + y.x, x.y + y.y);
  }
}

// sqrt(2) sqrt(W) (phase-factored): x' = x + e^{-3 i pi/4} y,
// y' = e^{-i pi/4} x + y; (-1 - i) y = (Im y - Re y) - i (Re y + Im y) and
// (1 - i) x = (Re x + Im x) + i (Im x - Re x), each scaled by 1/sqrt(2)
template <int NR, int B>
__device__ __forceinline__ void rg_hw1(c128 (&a)[NR]) {
  constexpr double h = 0.70710678118654752440;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    const c128 x = a[j], y = a[k];
    a[j] = make_double2(fma(h, y.y - y.x, x.x), fma(-h, y.x + y.y, x.y));
    a[k] = make_double2(fma(h, x.x + x.y, y.x), fma(h, x.y - x.x, y.y));
  }
}

// Rx-type [[C, -iS], [-iS, C]]: (Re x, Im y) rotate by p, (Im x, Re y) by -p
template <int NR, int B, bool ADJ, bool N0>
__device__ __forceinline__ void rg_sxr1(c128 (&a)[NR], const SRec &r) {
  const double al = ADJ ? -r.ab[0] : r.ab[0], be = ADJ ? -r.ab[1] : r.ab[1];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    shr<N0>(a[j].x, a[k].y, al, be);
    shr<N0>(a[j].y, a[k].x, -al, -be);
  }
}

// Ry-type real rotation of (x, y), real and imaginary parts alike
template <int NR, int B, bool ADJ, bool N0>
__device__ __forceinline__ void rg_srr1(c128 (&a)[NR], const SRec &r) {
  const double al = ADJ ? -r.ab[0] : r.ab[0], be = ADJ ? -r.ab[1] : r.ab[1];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    shr<N0>(a[j].x, a[k].x, al, be);
    shr<N0>(a[j].y, a[k].y, al, be);
  }
}

// diag(1, e^{ip}): the |1> amplitudes rotate in the complex plane
template <int NR, int B, bool ADJ, bool N0>
__device__ __forceinline__ void rg_sph1(c128 (&a)[NR], const SRec &r) {
  const double al = ADJ ? -r.ab[0] : r.ab[0], be = ADJ ? -r.ab[1] : r.ab[1];
#pragma unroll
  for (int j = 0; j < NR; j++)
    if ((j >> B) & 1) shr<N0>(a[j].x, a[j].y, al, be);
}

// diag(e^{ip0}, e^{ip1})
template <int NR, int B, bool ADJ, bool N0, bool N1>
__device__ __forceinline__ void rg_sdg1(c128 (&a)[NR], const SRec &r) {
  const double a0 = ADJ ? -r.ab[0] : r.ab[0], b0 = ADJ ? -r.ab[1] : r.ab[1];
  const double a1 = ADJ ? -r.ab[2] : r.ab[2], b1 = ADJ ? -r.ab[3] : r.ab[3];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if ((j >> B) & 1) shr<N1>(a[j].x, a[j].y, a1, b1);
    else shr<N0>(a[j].x, a[j].y, a0, b0);
  }
}

// D^dagger R(p) D with D = diag(1, e^{i chi}): rotation 0 is chi (stored
// with C >= 0, never negated), rotation 1 is p; the adjoint negates p only
template <int NR, int B, bool ADJ, bool N1>
__device__ __forceinline__ void rg_srd1(c128 (&a)[NR], const SRec &r) {
  const double ac = r.ab[0], bc = r.ab[1];
  const double al = ADJ ? -r.ab[2] : r.ab[2], be = ADJ ? -r.ab[3] : r.ab[3];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    shr<false>(a[k].x, a[k].y, ac, bc);
    shr<N1>(a[j].x, a[k].x, al, be);
    shr<N1>(a[j].y, a[k].y, al, be);
    shr<false>(a[k].x, a[k].y, -ac, -bc);
  }
}

// fSim with Delta = 0: |01>,|10> block as an Rx-type rotation (rotation 0),
// e^{-i phi} on |11> (rotation 1)
template <int NR, int B0, int B1, bool ADJ, bool N0, bool N1>
__device__ __forceinline__ void rg_sfx(c128 (&a)[NR], const SRec &r) {
  const double a0 = ADJ ? -r.ab[0] : r.ab[0], b0 = ADJ ? -r.ab[1] : r.ab[1];
  const double a1 = ADJ ? -r.ab[2] : r.ab[2], b1 = ADJ ? -r.ab[3] : r.ab[3];
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    const int i1 = j | (1 << B0), i2 = j | (1 << B1), i3 = i1 | i2;
    shr<N0>(a[i1].x, a[i2].y, a0, b0);
    shr<N0>(a[i1].y, a[i2].x, -a0, -b0);
    shr<N1>(a[i3].x, a[i3].y, a1, b1);
  }
}

// Re sum conj(b) (D a) over the groups of an op (gradient inner products)
template <int NR, int B>
__device__ __forceinline__ double gr_dense1(const c128 (&a)[NR], const c128 (&b)[NR], cmat *D) {
  const c128 d00 = tc(D[0]), d01 = tc(D[1]), d10 = tc(D[2]), d11 = tc(D[3]);
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    acc += redot(b[j], cfma(d00, a[j], cmul(d01, a[k])));
    acc += redot(b[k], cfma(d10, a[j], cmul(d11, a[k])));
  }
  return acc;
}

template <int NR, int B>
__device__ __forceinline__ double gr_diag1(const c128 (&a)[NR], const c128 (&b)[NR], cmat *D) {
  const c128 d0 = tc(D[0]), d1 = tc(D[3]);
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) acc += redot(b[j], cmul((j >> B) & 1 ? d1 : d0, a[j]));
  return acc;
}

template <int NR, int B0, int B1>
__device__ __forceinline__ double gr_dense2(const c128 (&a)[NR], const c128 (&b)[NR], cmat *D) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    int idx[4];
#pragma unroll
    for (int l = 0; l < 4; l++) idx[l] = j | ((l & 1) << B0) | ((l >> 1) << B1);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      c128 w = cmul(tc(D[r * 4 + 0]), a[idx[0]]);
      w = cfma(tc(D[r * 4 + 1]), a[idx[1]], w);
      w = cfma(tc(D[r * 4 + 2]), a[idx[2]], w);
      w = cfma(tc(D[r * 4 + 3]), a[idx[3]], w);
      acc += redot(b[idx[r]], w);
    }
  }
  return acc;
}

template <int NR>
__device__ __forceinline__ double gr_dense4(const c128 (&a)[NR], const c128 (&b)[NR], cmat *D) {
  double acc = 0.0;
  if constexpr (NR == 16) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
      c128 w = cmul(tc(D[r * 16]), a[0]);
#pragma unroll
      for (int c = 1; c < 16; c++) w = cfma(tc(D[r * 16 + c]), a[c], w);
      acc += redot(b[r], w);
    }
  }
  return acc;
}

// Im<b| G |a> / 2 for G = X, Y or Z on register bit B (a is Phi after the op)
template <int NR, int B, int GEN>
__device__ __forceinline__ double gr_gen(const c128 (&a)[NR], const c128 (&b)[NR]) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & (1 << B)) continue;
    const int k = j | (1 << B);
    if (GEN == GK_GENZ) {
      // Im(conj(b_j) a_j) - Im(conj(b_k) a_k)
      acc = fma(b[j].x, a[j].y, acc);
      acc = fma(-b[j].y, a[j].x, acc);
      acc = fma(-b[k].x, a[k].y, acc);
      acc = fma(b[k].y, a[k].x, acc);
    } else if (GEN == GK_GENX) {
      // Im(conj(b_j) a_k) + Im(conj(b_k) a_j)
      acc = fma(b[j].x, a[k].y, acc);
      acc = fma(-b[j].y, a[k].x, acc);
      acc = fma(b[k].x, a[j].y, acc);
      acc = fma(-b[k].y, a[j].x, acc);
    } else {
      // (Y a)_j = -i a_k, (Y a)_k = i a_j: Re(conj(b_k) a_j) - Re(conj(b_j) a_k)
      acc = fma(b[k].x, a[j].x, acc);
      acc = fma(b[k].y, a[j].y, acc);
      acc = fma(-b[j].x, a[k].x, acc);
      acc = fma(-b[j].y, a[k].y, acc);
    }
  }
  return 0.5 * acc;
}

// dispatch on kind and register bits (compile-time bit positions keep the
// amplitude array in VGPRs)
#define VQC_CASE1(FN, B) \
  case B:                \
    if constexpr (B < R) FN<NR, B, ADJ>(a, M); \
    break;
#define VQC_CASE2(FN, B0, B1) \
  case B0 * 4 + B1:           \
    if constexpr (B0 < R && B1 < R) FN<NR, B0, B1, ADJ>(a, M); \
    break;
#define VQC_SWITCH2(FN)                                                         \
  switch (g.r[0] * 4 + g.r[1]) {                                               \
    VQC_CASE2(FN, 0, 1) VQC_CASE2(FN, 0, 2) VQC_CASE2(FN, 0, 3)                \
    VQC_CASE2(FN, 1, 0) VQC_CASE2(FN, 1, 2) VQC_CASE2(FN, 1, 3)                \
    VQC_CASE2(FN, 2, 0) VQC_CASE2(FN, 2, 1) VQC_CASE2(FN, 2, 3)                \
    VQC_CASE2(FN, 3, 0) VQC_CASE2(FN, 3, 1) VQC_CASE2(FN, 3, 2)                \
    default: break;                                                            \
  }

// rotation kinds on one register bit B: kind x bit x negation bits
template <int R, bool ADJ, int B>
__device__ __forceinline__ void rg_s1_at(c128 (&a)[1 << R], int kind, const SRec &r) {
  constexpr int NR = 1 << R;
  if constexpr (B < R) {
    const uint32_t n = r.neg;
    switch (kind) {
      case GK_SXR1:
        if (n & 1) rg_sxr1<NR, B, ADJ, true>(a, r); else rg_sxr1<NR, B, ADJ, false>(a, r);
        break;
      case GK_SRR1:
        if (n & 1) rg_srr1<NR, B, ADJ, true>(a, r); else rg_srr1<NR, B, ADJ, false>(a, r);
        break;
      case GK_SPH1:
        if (n & 1) rg_sph1<NR, B, ADJ, true>(a, r); else rg_sph1<NR, B, ADJ, false>(a, r);
        break;
      case GK_SDG1:
        switch (n & 3) {
          case 0: rg_sdg1<NR, B, ADJ, false, false>(a, r); break;
          case 1: rg_sdg1<NR, B, ADJ, true, false>(a, r); break;
          case 2: rg_sdg1<NR, B, ADJ, false, true>(a, r); break;
          default: rg_sdg1<NR, B, ADJ, true, true>(a, r); break;
        }
        break;
      default:  // GK_SRD1
        if (n & 2) rg_srd1<NR, B, ADJ, true>(a, r); else rg_srd1<NR, B, ADJ, false>(a, r);
        break;
    }
  }
}

template <int R, bool ADJ>
__device__ __forceinline__ void rg_apply_s1(c128 (&a)[1 << R], const DGate &g, const SRec &r) {
  switch (g.r[0]) {
    case 0: rg_s1_at<R, ADJ, 0>(a, g.kind, r); break;
    case 1: rg_s1_at<R, ADJ, 1>(a, g.kind, r); break;
    case 2: rg_s1_at<R, ADJ, 2>(a, g.kind, r); break;
    default: rg_s1_at<R, ADJ, 3>(a, g.kind, r); break;
  }
}

template <int R, bool ADJ, int B0, int B1>
__device__ __forceinline__ void rg_sfx_at(c128 (&a)[1 << R], const SRec &r) {
  constexpr int NR = 1 << R;
  if constexpr (B0 < R && B1 < R && B0 != B1) {
    switch (r.neg & 3) {
      case 0: rg_sfx<NR, B0, B1, ADJ, false, false>(a, r); break;
      case 1: rg_sfx<NR, B0, B1, ADJ, true, false>(a, r); break;
      case 2: rg_sfx<NR, B0, B1, ADJ, false, true>(a, r); break;
      default: rg_sfx<NR, B0, B1, ADJ, true, true>(a, r); break;
    }
  }
}

template <int R, bool ADJ>
__device__ __forceinline__ void rg_apply_sfx(c128 (&a)[1 << R], const DGate &g, const SRec &r) {
  switch (g.r[0] * 4 + g.r[1]) {
    case 1: rg_sfx_at<R, ADJ, 0, 1>(a, r); break;
    case 2: rg_sfx_at<R, ADJ, 0, 2>(a, r); break;
    case 3: rg_sfx_at<R, ADJ, 0, 3>(a, r); break;
    case 4: rg_sfx_at<R, ADJ, 1, 0>(a, r); break;
    case 6: rg_sfx_at<R, ADJ, 1, 2>(a, r); break;
    case 7: rg_sfx_at<R, ADJ, 1, 3>(a, r); break;
    case 8: rg_sfx_at<R, ADJ, 2, 0>(a, r); break;
    case 9: rg_sfx_at<R, ADJ, 2, 1>(a, r); break;
    case 11: rg_sfx_at<R, ADJ, 2, 3>(a, r); break;
    case 12: rg_sfx_at<R, ADJ, 3, 0>(a, r); break;
    case 13: rg_sfx_at<R, ADJ, 3, 1>(a, r); break;
    default: rg_sfx_at<R, ADJ, 3, 2>(a, r); break;
  }
}

// D4: whether 16x16 superoperators can occur (vectorised density matrices);
// the pure-state LDS kernels leave them out, which frees registers
template <int R, bool ADJ, bool D4>
__device__ __forceinline__ void rg_apply_generic(c128 (&a)[1 << R], const DGate &g, cmat *M) {
  constexpr int NR = 1 << R;
  switch (g.kind) {
    case GK_DENSE1:
      switch (g.r[0]) { VQC_CASE1(rg_dense1, 0) VQC_CASE1(rg_dense1, 1) VQC_CASE1(rg_dense1, 2) VQC_CASE1(rg_dense1, 3) default: break; }
      break;
    case GK_DIAG1:
      switch (g.r[0]) { VQC_CASE1(rg_diag1, 0) VQC_CASE1(rg_diag1, 1) VQC_CASE1(rg_diag1, 2) VQC_CASE1(rg_diag1, 3) default: break; }
      break;
    case GK_XROT1:
      switch (g.r[0]) { VQC_CASE1(rg_xrot1, 0) VQC_CASE1(rg_xrot1, 1) VQC_CASE1(rg_xrot1, 2) VQC_CASE1(rg_xrot1, 3) default: break; }
      break;
    case GK_REAL1:
      switch (g.r[0]) { VQC_CASE1(rg_real1, 0) VQC_CASE1(rg_real1, 1) VQC_CASE1(rg_real1, 2) VQC_CASE1(rg_real1, 3) default: break; }
      break;
    case GK_RDIAG1:
      switch (g.r[0]) { VQC_CASE1(rg_rdiag1, 0) VQC_CASE1(rg_rdiag1, 1) VQC_CASE1(rg_rdiag1, 2) VQC_CASE1(rg_rdiag1, 3) default: break; }
      break;
    case GK_PHASE1:
      switch (g.r[0]) { VQC_CASE1(rg_phase1, 0) VQC_CASE1(rg_phase1, 1) VQC_CASE1(rg_phase1, 2) VQC_CASE1(rg_phase1, 3) default: break; }
      break;
    case GK_FSIMX: VQC_SWITCH2(rg_fsimx) break;
    case GK_DENSE2: VQC_SWITCH2(rg_dense2) break;
    case GK_DIAG2: VQC_SWITCH2(rg_diag2) break;
    case GK_FSIM: VQC_SWITCH2(rg_fsim) break;
    case GK_CX:
      switch (g.r[0] * 4 + g.r[1]) {
#define VQC_CASECX(B0, B1) \
  case B0 * 4 + B1:        \
    if constexpr (B0 < R && B1 < R) rg_cx<NR, B0, B1>(a); \
    break;
        VQC_CASECX(0, 1) VQC_CASECX(0, 2) VQC_CASECX(0, 3) VQC_CASECX(1, 0) VQC_CASECX(1, 2)
        VQC_CASECX(1, 3) VQC_CASECX(2, 0) VQC_CASECX(2, 1) VQC_CASECX(2, 3) VQC_CASECX(3, 0)
        VQC_CASECX(3, 1) VQC_CASECX(3, 2)
#undef VQC_CASECX
        default: break;
      }
      break;
    case GK_DENSE3: {
      int rm[8];
      switch (dense3_map(g.r[0], g.r[1], g.r[2], rm)) {
        case 7: rg_dense3<NR, 0, 1, 2, ADJ>(a, M, rm); break;
        case 11: if constexpr (R > 3) rg_dense3<NR, 0, 1, 3, ADJ>(a, M, rm); break;
        case 13: if constexpr (R > 3) rg_dense3<NR, 0, 2, 3, ADJ>(a, M, rm); break;
        case 14: if constexpr (R > 3) rg_dense3<NR, 1, 2, 3, ADJ>(a, M, rm); break;
        default: break;
      }
      break;
    }
    case GK_DENSE4:
      if constexpr (D4) rg_dense4<NR, ADJ>(a, M);
      break;
    case GK_DEPOL4:
      if constexpr (D4) rg_depol4<NR>(a, M);
      break;
    default: break;
  }
}

// move t[j] into the register that holds a[j] (the asm ties the result to
// a[j]'s register)
__device__ __forceinline__ void tied_set(double &d, double s) { asm("v_mov_b64 %0, %1" : "+v"(d) : "v"(s)); }

// Apply one op to the lane's amplitudes.  The op loop keeps the amplitudes
// in fixed registers: rotation kinds update them in place; every other kind
// works on a copy whose results are moved back with register-tied moves, so
// no dispatch arm leaves a value in another register (which would make the
// register allocator copy all amplitudes after every op).
template <int R, bool ADJ, bool D4 = true>
__device__ __forceinline__ void rg_apply_pre(c128 (&a)[1 << R], const DGate &g, const SRec &rec, cmat *mats) {
  constexpr int NR = 1 << R;
  cmat *M = mats + g.mat;
  const int kind = g.kind;
  if (kind >= GK_SXR1 && kind <= GK_SFX) {
    if (kind == GK_SFX) rg_apply_sfx<R, ADJ>(a, g, rec);
    else rg_apply_s1<R, ADJ>(a, g, rec);
    return;
  }
  if (kind == GK_NONE) return;
  c128 t[NR];
#pragma unroll
  for (int j = 0; j < NR; j++) t[j] = a[j];
  rg_apply_generic<R, ADJ, D4>(t, g, M);
#pragma unroll
  for (int j = 0; j < NR; j++) {
    tied_set(a[j].x, t[j].x);
    tied_set(a[j].y, t[j].y);
  }
}


// one op from its program entry
template <int R, bool ADJ, bool D4 = true>
__device__ __forceinline__ void rg_apply_op(c128 (&a)[1 << R], const DOp &E, cmat *mats) {
  SRec r;
  r.neg = E.neg;
  r.pad = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) r.ab[i] = E.ab[i];
#pragma unroll
  for (int i = 4; i < 7; i++) r.ab[i] = 0.0;
  rg_apply_pre<R, ADJ, D4>(a, E.g, r, mats);
}

// wait for all outstanding scalar (and LDS) loads.  Scalar loads may return
// out of order, so a wait for one of them is a wait for all: the op loops
// wait explicitly for the op about to run *before* issuing the load of the
// next one, which then overlaps the current op's FP64 work.
__device__ __forceinline__ void lgkm_wait() { __builtin_amdgcn_s_waitcnt(0xc07f); }

// Ops g0 .. g1-1 of a program in order (prog[g] is op g; prog[g1] is
// readable: the next stage's op or padding).  The entry of op g + 1 is in
// flight while op g runs.
template <int R, bool D4 = true>
__device__ __forceinline__ void rg_run(c128 (&a)[1 << R], const DOp *prog, int g0, int g1, cmat *mats) {
  if (g0 >= g1) return;
  DOp A = ldc(&prog[g0]);
  for (int g = g0; g < g1; g++) {
    lgkm_wait();
    const DOp B = ldc(&prog[g + 1]);
    rg_apply_op<R, false, D4>(a, A, mats);
    A = B;
  }
}

#define VQC_GCASE1(FN, B) \
  case B:                 \
    if constexpr (B < R) v = FN<NR, B>(a, b, D); \
    break;
#define VQC_GCASE2(B0, B1) \
  case B0 * 4 + B1:        \
    if constexpr (B0 < R && B1 < R) v = gr_dense2<NR, B0, B1>(a, b, D); \
    break;

template <int R, int B>
__device__ __forceinline__ double rg_grad_gen_at(const c128 (&a)[1 << R], const c128 (&b)[1 << R], int kind) {
  if constexpr (B < R) {
    if (kind == GK_GENZ) return gr_gen<1 << R, B, GK_GENZ>(a, b);
    if (kind == GK_GENX) return gr_gen<1 << R, B, GK_GENX>(a, b);
    return gr_gen<1 << R, B, GK_GENY>(a, b);
  }
  return 0.0;
}

template <int R>
__device__ __forceinline__ double rg_grad_gen(const c128 (&a)[1 << R], const c128 (&b)[1 << R], int kind, int r0) {
  switch (r0) {
    case 0: return rg_grad_gen_at<R, 0>(a, b, kind);
    case 1: return rg_grad_gen_at<R, 1>(a, b, kind);
    case 2: return rg_grad_gen_at<R, 2>(a, b, kind);
    default: return rg_grad_gen_at<R, 3>(a, b, kind);
  }
}

// derivative records reuse the register bits of their op
template <int R, bool D4 = true>
__device__ __forceinline__ double rg_grad(const c128 (&a)[1 << R], const c128 (&b)[1 << R], const DGate &g,
                                          const DDeriv &d, cmat *mats) {
  constexpr int NR = 1 << R;
  cmat *D = mats + d.mat;
  double v = 0.0;
  switch (d.kind) {
    case GK_DENSE1:
      switch (g.r[0]) { VQC_GCASE1(gr_dense1, 0) VQC_GCASE1(gr_dense1, 1) VQC_GCASE1(gr_dense1, 2) VQC_GCASE1(gr_dense1, 3) default: break; }
      break;
    case GK_DIAG1:
      switch (g.r[0]) { VQC_GCASE1(gr_diag1, 0) VQC_GCASE1(gr_diag1, 1) VQC_GCASE1(gr_diag1, 2) VQC_GCASE1(gr_diag1, 3) default: break; }
      break;
    case GK_DENSE2:
      switch (g.r[0] * 4 + g.r[1]) {
        VQC_GCASE2(0, 1) VQC_GCASE2(0, 2) VQC_GCASE2(0, 3) VQC_GCASE2(1, 0) VQC_GCASE2(1, 2) VQC_GCASE2(1, 3)
        VQC_GCASE2(2, 0) VQC_GCASE2(2, 1) VQC_GCASE2(2, 3) VQC_GCASE2(3, 0) VQC_GCASE2(3, 1) VQC_GCASE2(3, 2)
        default: break;
      }
      break;
    case GK_DENSE4:
      if constexpr (D4) v = gr_dense4<NR>(a, b, D);
      break;
    case GK_GENX: case GK_GENY: case GK_GENZ:
      v = rg_grad_gen<R>(a, b, d.kind, g.r[0]);
      break;
    default: break;
  }
  return v;
}

// one DPP move of a double (both halves) from the lane the control selects;
// lanes in rows outside ROWMASK get 0
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, false);
  const int rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(rhi, rlo);
}

// Sum over the lanes of a wave (W lanes active, W a power of two).  A full
// wave64 reduces with DPP moves (quad swaps, half-row and row mirrors, then
// the row-15 and row-31 broadcasts), all in the VALU, and the total is read
// from lane 63 into a scalar; narrower groups use lane shuffles.  The result
// is the same in every lane.
// the sum over a wave of W lanes, valid in lane W - 1 (all lanes for W < 64)
template <int W>
__device__ __forceinline__ double wave_sum_last(double v) {
  if constexpr (W == 64) {
    v += dpp_d<0xB1>(v);        // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);        // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);       // row_half_mirror: sum of 8
    v += dpp_d<0x140>(v);       // row_mirror: sum of 16
    v += dpp_d<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
    v += dpp_d<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3: lane 63 = total
    return v;
  } else {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
  }
}

template <int W>
__device__ __forceinline__ double wave_sum(double v) {
  if constexpr (W == 64) {
    v += dpp_d<0xB1>(v);        // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);        // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);       // row_half_mirror: sum of 8
    v += dpp_d<0x140>(v);       // row_mirror: sum of 16
    v += dpp_d<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
    v += dpp_d<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3: lane 63 = total
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
  } else {
#pragma unroll
    for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
    return v;
  }
}

// tile-local bit -> global qubit for a runtime (uniform) local bit: one
// scalar dword load from the pass table instead of indexing a local copy,
// which would force the copy into scratch memory
__device__ __forceinline__ int tq_at(const DPass *gp, int idx) {
  const uint32_t w = *((const VQC_AS_CONST uint32_t *)gp->tq + (idx >> 2));
  return (w >> (8 * (idx & 3))) & 0xff;
}

template <typename JT>
__device__ __forceinline__ int find_job(const JT *__restrict__ jobs, int n_jobs, int64_t u) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ldc(&jobs[mid].unit0) <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ fused LDS pass

// MODE bit 0: the adjoint step; bit 1: 16x16 superoperators compiled in
// (density matrices), whose adjoint takes M^{-1} for non-unitary ops
template <int K, int R, int MODE>
__global__ void __launch_bounds__(1 << (K - R))
k_pass_lds(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units, DOverride ov) {
  constexpr bool ADJ = (MODE & 1) != 0;
  constexpr bool D4 = (MODE & 2) != 0;
  constexpr int T = 1 << (K - R);
  constexpr int NR = 1 << R;
  constexpr int WS = T < 64 ? T : 64;
  constexpr int NW = (T + 63) / 64;
  extern __shared__ c128 smem[];
  __shared__ double red[ADJ ? kMaxVarPerPass : 1][NW];
  c128 *la = smem;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;

  // The forward loads its tile into registers first.  With a persistent grid
  // (a grid size below the tile count, vqc_tune.grid_blocks) each block also
  // prefetches its next tile during the current tile's stages; by default the
  // grid has one block per tile and the hardware overlaps the blocks' memory
  // and FP64 phases (measured faster than persistent prefetching).
  [[maybe_unused]] c128 pf[NR];
  [[maybe_unused]] bool have_pf = false;
  auto tile_addr = [&](int64_t uu, const DJob &JJ, const DPass &PQ, uint64_t &gb0, uint64_t &st0) {
    uint64_t g0 = (uint64_t)(uu - JJ.unit0);
#pragma unroll
    for (int i = 0; i < K; i++) g0 = ins0<uint64_t>(g0, PQ.tq[i]);
    uint64_t s0 = 0;
#pragma unroll
    for (int i = 0; i < K - R; i++) s0 |= (uint64_t)((t >> i) & 1) << PQ.tq[i];
    gb0 = g0;
    st0 = s0;
  };
  auto prefetch = [&](int64_t uu) {
    const DJob JN = ldc(&jobs[find_job(jobs, n_jobs, uu)]);
    const DPass PN = ldc(JN.pass);
    const gc128 *srcn = (const gc128 *)(ov.use ? ov.a : JN.a);
    uint64_t g0, s0;
    tile_addr(uu, JN, PN, g0, s0);
#pragma unroll
    for (int j = 0; j < NR; j++) {
      uint64_t oj = 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if ((j >> i) & 1) oj |= 1ull << PN.tq[K - R + i];
      pf[j] = ldg(&srcn[g0 | s0 | oj]);
    }
  };
  if constexpr (!ADJ) {
    if ((int64_t)blockIdx.x < total_units) {
      prefetch(blockIdx.x);
      have_pf = true;
    }
  }
  for (int64_t u = blockIdx.x; u < total_units; u += gridDim.x) {
    const DJob J = ldc(&jobs[find_job(jobs, n_jobs, u)]);
    const DPass PP = ldc(J.pass);
    const DPass *P = &PP;
    const int64_t tile = u - J.unit0;
    gc128 *A = (gc128 *)(ov.use ? ov.a : J.a);
    gc128 *Bv = (gc128 *)(ov.use ? ov.b : J.b);
    cmat *MT = (cmat *)(ov.use ? ov.mats : J.mats);
    const DOp *prog = (const DOp *)(MT + P->prog) + 1;
    double *PT = ov.use ? ov.partials : J.partials;
    const int mode = ov.use ? ov.mode : J.mode;
    uint64_t gbase = (uint64_t)tile;
#pragma unroll
    for (int i = 0; i < K; i++) gbase = ins0<uint64_t>(gbase, P->tq[i]);
    uint64_t st = 0;
#pragma unroll
    for (int i = 0; i < K - R; i++) st |= (uint64_t)((t >> i) & 1) << P->tq[i];
    const gc128 *src = A;
    [[maybe_unused]] const gc128 *srcb = Bv;
    gc128 *dst = A;
    [[maybe_unused]] gc128 *dstb = Bv;
    if (mode == 1) {
      if constexpr (ADJ) {
        dst = (gc128 *)(ov.use ? ov.a2 : J.a2);
        dstb = (gc128 *)(ov.use ? ov.b2 : J.b2);
      } else {
        dst = Bv;
      }
    }
    const int nst = P->nst;
    // direct HBM access for the first / last stage in execution order
    const bool din = ADJ ? (P->lowfree >> 1) & 1 : false;
    const bool dout = ADJ ? P->lowfree & 1 : (P->lowfree >> 1) & 1;
    // LDS -> HBM in the pass's output layout (the input layout unless the
    // pass moves qubits): lanes run over the output's lowest tile bits
    auto store_out = [&](const c128 *lx, gc128 *d) {
      uint64_t gbo = (uint64_t)tile;
#pragma unroll
      for (int i = 0; i < K; i++) gbo = ins0<uint64_t>(gbo, P->tqo[i]);
      uint64_t so = 0;
      int sl = 0;
#pragma unroll
      for (int i = 0; i < K - R; i++)
        if ((t >> i) & 1) {
          so |= 1ull << P->tqo[i];
          sl |= 1 << P->lbo[i];
        }
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t oj = 0;
        int ol = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) {
            oj |= 1ull << P->tqo[K - R + i];
            ol |= 1 << P->lbo[K - R + i];
          }
        stg(&d[gbo | so | oj], lx[swz(sl | ol)]);
      }
    };
    // HBM -> LDS, coalesced over the low tile bits
    auto load_in = [&](c128 *lx, const gc128 *sp) {
#pragma unroll
      for (int j = 0; j < NR; j++) {
        uint64_t oj = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) oj |= 1ull << P->tq[K - R + i];
        lx[swz(j * T + t)] = ldg(&sp[gbase | st | oj]);
      }
    };
    if constexpr (!ADJ) {
      // the tile was prefetched by the previous iteration (or before the loop)
#pragma unroll
      for (int j = 0; j < NR; j++) la[swz(j * T + t)] = pf[j];
      const int64_t un = u + gridDim.x;
      if (un < total_units) prefetch(un);
      __syncthreads();
      for (int s = 0; s < nst; s++) {
        const DStage S = ldc(&P->stages[s]);
        int base = t;
#pragma unroll
        for (int i = 0; i < R; i++) base = ins0<int>(base, S.srt[i]);
        int lo[NR];
#pragma unroll
        for (int j = 0; j < NR; j++) {
          int o = 0;
#pragma unroll
          for (int i = 0; i < R; i++)
            if ((j >> i) & 1) o |= 1 << S.rbit[i];
          lo[j] = o;
        }
        const bool last = (s == nst - 1) && dout;
        c128 a[NR];
#pragma unroll
        for (int j = 0; j < NR; j++) a[j] = la[swz(base | lo[j])];
        rg_run<R, D4>(a, prog, S.g0, S.g1, MT);
        if (last) {
          // HBM address of local index base | lo[j]: gbase + scatter(base) + scatter(lo[j])
          uint64_t gb = gbase;
#pragma unroll
          for (int i = 0; i < K; i++)
            if ((base >> i) & 1) gb |= 1ull << P->tq[i];
#pragma unroll
          for (int j = 0; j < NR; j++) {
            uint64_t go = 0;
#pragma unroll
            for (int i = 0; i < R; i++)
              if ((j >> i) & 1) go |= 1ull << tq_at(J.pass, S.rbit[i]);
            stg(&dst[gb | go], a[j]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < NR; j++) la[swz(base | lo[j])] = a[j];
          __syncthreads();
        }
      }
      if (!dout) store_out(la, dst);
    } else {
      // Phi and Psi share the one LDS tile: every change of layout moves Phi
      // through it, then Psi (half the LDS of two tiles, so twice the
      // resident blocks, for two more barriers per stage change).  Registers
      // a, b carry a stage's amplitudes into the next; pb / plo: the layout
      // Psi waits in until the next stage's read.
      c128 a[NR], b[NR];
      int pb = 0, plo[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) plo[j] = 0;
      if (!din) load_in(la, src);
      __syncthreads();
      for (int si = 0; si < nst; si++) {
        const int s = nst - 1 - si;
        const DStage S = ldc(&P->stages[s]);
        int base = t;
#pragma unroll
        for (int i = 0; i < R; i++) base = ins0<int>(base, S.srt[i]);
        int lo[NR];
#pragma unroll
        for (int j = 0; j < NR; j++) {
          int o = 0;
#pragma unroll
          for (int i = 0; i < R; i++)
            if ((j >> i) & 1) o |= 1 << S.rbit[i];
          lo[j] = o;
        }
        const bool first = (si == 0) && din, last = (si == nst - 1) && dout;
        uint64_t gb = 0;
        if (first || last) {
          gb = gbase;
#pragma unroll
          for (int i = 0; i < K; i++)
            if ((base >> i) & 1) gb |= 1ull << P->tq[i];
        }
        if (first) {
#pragma unroll
          for (int j = 0; j < NR; j++) {
            uint64_t go = 0;
#pragma unroll
            for (int i = 0; i < R; i++)
              if ((j >> i) & 1) go |= 1ull << tq_at(J.pass, S.rbit[i]);
            a[j] = ldg(&src[gb | go]);
            b[j] = ldg(&srcb[gb | go]);
          }
        } else {
          // Phi is in the tile (loaded, or written by the previous stage)
#pragma unroll
          for (int j = 0; j < NR; j++) a[j] = la[swz(base | lo[j])];
          __syncthreads();
          if (si == 0) {
            load_in(la, srcb);
          } else {
#pragma unroll
            for (int j = 0; j < NR; j++) la[swz(pb | plo[j])] = b[j];
          }
          __syncthreads();
#pragma unroll
          for (int j = 0; j < NR; j++) b[j] = la[swz(base | lo[j])];
        }
        DOp E = ldc(&prog[S.g1 - 1]);
        for (int g = S.g1 - 1; g >= S.g0; g--) {
          lgkm_wait();
          const DOp En = ldc(&prog[g - 1]);  // prog[g0 - 1] is readable
          const int nd = E.g.nd & 0xff;
          auto grads = [&]() {  // Re<Psi| dQ |Phi before Q>
            if (E.pad >> 31) {  // one generator derivative, carried in the entry
              const double v = wave_sum<WS>(rg_grad_gen<R>(a, b, E.pad & 0xff, E.g.r[0]));
              if (lane == 0) red[(E.pad >> 8) & 0xffff][wave] = v;
              return;
            }
            for (int d = 0; d < nd; d++) {
              const DDeriv Dd = ldc(&P->derivs[E.g.d0 + d]);
              double v = wave_sum<WS>(rg_grad<R, D4>(a, b, E.g, Dd, MT));
              if (lane == 0) red[Dd.local][wave] = v;
            }
          };
          // generator form (pure states only): Phi after Q; density
          // matrices keep one call site of the reductions (no spills)
          if (!D4 && (E.g.nd & kGenFlag)) grads();
          if (D4 && (E.g.nd & kInvFlag)) {  // Phi <- M^{-1} Phi (stored after M)
            DOp Ei = E;
            Ei.g.mat += (E.g.kind == GK_DENSE4 || E.g.kind == GK_DEPOL4) ? 256 : 16;
            rg_apply_op<R, false, D4>(a, Ei, MT);
          } else {
            rg_apply_op<R, true, D4>(a, E, MT);  // Phi <- Q^dagger Phi
          }
          if (D4 || !(E.g.nd & kGenFlag)) grads();
          rg_apply_op<R, true, D4>(b, E, MT);  // Psi <- Q^dagger Psi
          E = En;
        }
        if (last) {
#pragma unroll
          for (int j = 0; j < NR; j++) {
            uint64_t go = 0;
#pragma unroll
            for (int i = 0; i < R; i++)
              if ((j >> i) & 1) go |= 1ull << tq_at(J.pass, S.rbit[i]);
            stg(&dst[gb | go], a[j]);
            stg(&dstb[gb | go], b[j]);
          }
        } else {
          // Phi into the tile in this stage's layout (the slots this lane
          // read), Psi held back in registers until the next stage's read
#pragma unroll
          for (int j = 0; j < NR; j++) la[swz(base | lo[j])] = a[j];
          pb = base;
#pragma unroll
          for (int j = 0; j < NR; j++) plo[j] = lo[j];
          __syncthreads();
        }
      }
      if (nst == 0) {
        // a pass without ops only moves qubits
        store_out(la, dst);
        __syncthreads();
        load_in(la, srcb);
        __syncthreads();
        store_out(la, dstb);
      } else if (!dout) {
        store_out(la, dst);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NR; j++) la[swz(pb | plo[j])] = b[j];
        __syncthreads();
        store_out(la, dstb);
      }
    }
    if constexpr (ADJ) {
      // a last stage stored straight to HBM has no barrier after its
      // reductions: wait for every wave's entries before summing them
      if (dout) __syncthreads();
      const int nv = P->nvar;
      for (int v = t; v < nv; v += T) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++) s += red[v][w];
        PT[(int64_t)ldc(&P->vslot[v]) * J.n_units + tile] = s;
      }
    }
    __syncthreads();
  }
}


// ------------------------------------------------------- register-only pass
// Each lane owns one tile of 2^R amplitudes (the stage's register bits); a
// block covers 256 tiles.  MODE 0: forward (in place, or out of place into
// J.b); MODE 1: noiseless adjoint (Alg. 2: Phi uncomputed in J.a, Psi in J.b);
// MODE 2: noisy adjoint (Sec. 3.5): J.a holds Phi at the pass start and is
// only read; Phi before each op is recomputed in registers, Psi <- M^dagger Psi.
// MODE 3: noisy adjoint in the inverse form (Alg. 2 applied to channels):
// Phi <- M^{-1} Phi in place (the inverse superoperator is stored right after
// M for ops flagged kInvFlag; other ops are unitary and use M^dagger), then
// the derivative reductions, then Psi <- M^dagger Psi.

template <int R, int MODE>
__global__ void __launch_bounds__(256) k_pass_reg(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units, DOverride ov) {
  constexpr int NR = 1 << R;
  __shared__ double red[MODE ? kMaxVarPerPass : 1][4];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  for (int64_t u = blockIdx.x; u < total_units; u += gridDim.x) {
    const DJob J = ldc(&jobs[find_job(jobs, n_jobs, u)]);
    const DPass PP = ldc(J.pass);
    const DPass *P = &PP;
    const int64_t ublk = u - J.unit0;
    gc128 *A = (gc128 *)(ov.use ? ov.a : J.a);
    gc128 *Bv = (gc128 *)(ov.use ? ov.b : J.b);
    cmat *MT = (cmat *)(ov.use ? ov.mats : J.mats);
    const DOp *prog = (const DOp *)(MT + P->prog) + 1;
    double *PT = ov.use ? ov.partials : J.partials;
    const int mode = ov.use ? ov.mode : J.mode;
    const int64_t tiles = (int64_t)1 << (J.nbits - R);
    const int64_t tile = ublk * 256 + t;
    const bool act = tile < tiles;
    const DStage S = ldc(&P->stages[0]);
    uint64_t base = act ? (uint64_t)tile : 0;
#pragma unroll
    for (int i = 0; i < R; i++) base = ins0<uint64_t>(base, P->tq[i]);
    uint64_t off[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) {
      uint64_t o = 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if ((j >> i) & 1) o |= 1ull << tq_at(J.pass, S.rbit[i]);
      off[j] = base | o;
    }
    c128 a[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) a[j] = act ? ldg(&A[off[j]]) : make_double2(0.0, 0.0);
    if constexpr (MODE == 0) {
      rg_run<R>(a, prog, S.g0, S.g1, MT);
      gc128 *dst = (mode == 1) ? Bv : A;
      if (act) {
#pragma unroll
        for (int j = 0; j < NR; j++) stg(&dst[off[j]], a[j]);
      }
    } else {
      c128 b[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) b[j] = act ? ldg(&Bv[off[j]]) : make_double2(0.0, 0.0);
      for (int g = S.g1 - 1; g >= S.g0; g--) {
        lgkm_wait();
        const DOp E = ldc(&prog[g]);
        const DGate &G = E.g;
        const int nd = G.nd & 0xff;
        const bool gen = G.nd & kGenFlag;
        if constexpr (MODE == 1 || MODE == 3) {
          auto grads = [&]() {
            if (E.pad >> 31) {  // one generator derivative, carried in the entry
              const double v = wave_sum<64>(rg_grad_gen<R>(a, b, E.pad & 0xff, G.r[0]));
              if (lane == 0) red[(E.pad >> 8) & 0xffff][wave] = v;
              return;
            }
            for (int d = 0; d < nd; d++) {
              const DDeriv Dd = ldc(&P->derivs[G.d0 + d]);
              const double v = wave_sum<64>(rg_grad<R>(a, b, G, Dd, MT));
              if (lane == 0) red[Dd.local][wave] = v;
            }
          };
          // generator form (pure states only): Phi after the op.  Mixed
          // circuits carry matrix derivatives only, and a second call site of
          // the reductions makes MODE 3 spill registers.
          if (MODE == 1 && gen) grads();
          if (MODE == 3 && (G.nd & kInvFlag)) {
            DOp Ei = E;
            Ei.g.mat += (G.kind == GK_DENSE4 || G.kind == GK_DEPOL4) ? 256 : 16;
            rg_apply_op<R, false>(a, Ei, MT);
          } else {
            rg_apply_op<R, true>(a, E, MT);
          }
          if (!gen) grads();
        } else {
          if (nd > 0) {
            // Phi before op g (after it, for generator derivatives),
            // recomputed from the pass-start checkpoint
            c128 c[NR];
#pragma unroll
            for (int j = 0; j < NR; j++) c[j] = a[j];
            rg_run<R>(c, prog, S.g0, gen ? g + 1 : g, MT);
            for (int d = 0; d < nd; d++) {
              const DDeriv Dd = ldc(&P->derivs[G.d0 + d]);
              const double v = wave_sum<64>(rg_grad<R>(c, b, G, Dd, MT));
              if (lane == 0) red[Dd.local][wave] = v;
            }
          }
        }
        rg_apply_op<R, true>(b, E, MT);
      }
      if (act) {
#pragma unroll
        for (int j = 0; j < NR; j++) {
          if constexpr (MODE == 1 || MODE == 3) stg(&A[off[j]], a[j]);
          stg(&Bv[off[j]], b[j]);
        }
      }
      __syncthreads();
      const int nv = P->nvar;
      for (int v = t; v < nv; v += 256)
        PT[(int64_t)ldc(&P->vslot[v]) * J.n_units + ublk] = (red[v][0] + red[v][1]) + (red[v][2] + red[v][3]);
    }
    __syncthreads();
  }
}


#ifndef __HIPCC_RTC__  // host launchers
}  // namespace vqc
#include <atomic>
namespace vqc {

// Per-device launch facts of one kernel instantiation, shared by every handle
// and stream of the process: whether the dynamic-LDS limit was raised and how
// many blocks the chip holds at once.  Racing first calls compute and store
// the same values (atomics, so no torn or unordered reads).
constexpr int kLaunchMaxDev = 64;
struct LaunchFacts {
  std::atomic<int> attr_set[kLaunchMaxDev];
  std::atomic<int> resident[kLaunchMaxDev];
};

template <int K, int R, int MODE>
hipError_t launch_lds_t(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                        hipStream_t st) {
  const size_t shmem = (size_t(1) << K) * sizeof(c128);  // the adjoint shares one tile between Phi and Psi
  static LaunchFacts facts;  // zero-initialised (static storage)
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kLaunchMaxDev) return hipErrorInvalidDevice;
  if (shmem > 65536 && !facts.attr_set[dev].load(std::memory_order_acquire)) {
    e = hipFuncSetAttribute((const void *)k_pass_lds<K, R, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
    if (e != hipSuccess) return e;
    facts.attr_set[dev].store(1, std::memory_order_release);
  }
  int g = grid;
  if (g <= 0) {
    // persistent grid: as many resident blocks as the chip holds
    int resident = facts.resident[dev].load(std::memory_order_acquire);
    if (!resident) {
      int per_cu = 0, cus = 0;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_pass_lds<K, R, MODE>, 1 << (K - R),
                                                       shmem);
      if (e != hipSuccess) return e;
      resident = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 256);
      facts.resident[dev].store(resident, std::memory_order_release);
    }
    g = (int)(total < resident ? total : resident);
  }
  hipLaunchKernelGGL((k_pass_lds<K, R, MODE>), dim3(g), dim3(1 << (K - R)), shmem, st, jobs, n_jobs, total, ov);
  return hipGetLastError();
}

template <int R, int MODE>
hipError_t launch_reg_t(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                        hipStream_t st) {
  const int g = grid > 0 ? grid : (int)(total < (1 << 30) ? total : (1 << 30));
  hipLaunchKernelGGL((k_pass_reg<R, MODE>), dim3(g), dim3(256), 0, st, jobs, n_jobs, total, ov);
  return hipGetLastError();
}

#endif  // __HIPCC_RTC__
}  // namespace vqc

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

// element (r, c) of M (row-major D x D) or of M^dagger
template <bool ADJ, int D>
__device__ __forceinline__ c128 mel(const c128 *__restrict__ M, int r, int c) {
  if (ADJ) return cconj(M[c * D + r]);
  return M[r * D + c];
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
__device__ __forceinline__ void rg_dense1(c128 (&a)[NR], const c128 *__restrict__ M) {
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
__device__ __forceinline__ void rg_diag1(c128 (&a)[NR], const c128 *__restrict__ M) {
  const c128 d0 = mel<ADJ, 2>(M, 0, 0), d1 = mel<ADJ, 2>(M, 1, 1);
#pragma unroll
  for (int j = 0; j < NR; j++) a[j] = cmul((j >> B) & 1 ? d1 : d0, a[j]);
}

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_dense2(c128 (&a)[NR], const c128 *__restrict__ M) {
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

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_diag2(c128 (&a)[NR], const c128 *__restrict__ M) {
  c128 d[4];
#pragma unroll
  for (int l = 0; l < 4; l++) d[l] = mel<ADJ, 4>(M, l, l);
#pragma unroll
  for (int j = 0; j < NR; j++) a[j] = cmul(d[((j >> B0) & 1) | (((j >> B1) & 1) << 1)], a[j]);
}

template <int NR, int B0, int B1, bool ADJ>
__device__ __forceinline__ void rg_fsim(c128 (&a)[NR], const c128 *__restrict__ M) {
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

template <int NR, bool ADJ>
__device__ __forceinline__ void rg_dense4(c128 (&a)[NR], const c128 *__restrict__ M) {
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

// Re sum conj(b) (D a) over the groups of an op (gradient inner products)
template <int NR, int B>
__device__ __forceinline__ double gr_dense1(const c128 (&a)[NR], const c128 (&b)[NR], const c128 *__restrict__ D) {
  const c128 d00 = D[0], d01 = D[1], d10 = D[2], d11 = D[3];
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
__device__ __forceinline__ double gr_diag1(const c128 (&a)[NR], const c128 (&b)[NR], const c128 *__restrict__ D) {
  const c128 d0 = D[0], d1 = D[3];
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) acc += redot(b[j], cmul((j >> B) & 1 ? d1 : d0, a[j]));
  return acc;
}

template <int NR, int B0, int B1>
__device__ __forceinline__ double gr_dense2(const c128 (&a)[NR], const c128 (&b)[NR], const c128 *__restrict__ D) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < NR; j++) {
    if (j & ((1 << B0) | (1 << B1))) continue;
    int idx[4];
#pragma unroll
    for (int l = 0; l < 4; l++) idx[l] = j | ((l & 1) << B0) | ((l >> 1) << B1);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      c128 w = cmul(D[r * 4 + 0], a[idx[0]]);
      w = cfma(D[r * 4 + 1], a[idx[1]], w);
      w = cfma(D[r * 4 + 2], a[idx[2]], w);
      w = cfma(D[r * 4 + 3], a[idx[3]], w);
      acc += redot(b[idx[r]], w);
    }
  }
  return acc;
}

template <int NR>
__device__ __forceinline__ double gr_dense4(const c128 (&a)[NR], const c128 (&b)[NR], const c128 *__restrict__ D) {
  double acc = 0.0;
  if constexpr (NR == 16) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
      c128 w = cmul(D[r * 16], a[0]);
#pragma unroll
      for (int c = 1; c < 16; c++) w = cfma(D[r * 16 + c], a[c], w);
      acc += redot(b[r], w);
    }
  }
  return acc;
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

template <int R, bool ADJ>
__device__ __forceinline__ void rg_apply(c128 (&a)[1 << R], const DGate &g, const c128 *__restrict__ mats) {
  constexpr int NR = 1 << R;
  const c128 *__restrict__ M = mats + g.mat;
  switch (g.kind) {
    case GK_DENSE1:
      switch (g.r[0]) { VQC_CASE1(rg_dense1, 0) VQC_CASE1(rg_dense1, 1) VQC_CASE1(rg_dense1, 2) VQC_CASE1(rg_dense1, 3) default: break; }
      break;
    case GK_DIAG1:
      switch (g.r[0]) { VQC_CASE1(rg_diag1, 0) VQC_CASE1(rg_diag1, 1) VQC_CASE1(rg_diag1, 2) VQC_CASE1(rg_diag1, 3) default: break; }
      break;
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
    case GK_DENSE4: rg_dense4<NR, ADJ>(a, M); break;
    default: break;
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

// derivative records reuse the register bits of their op
template <int R>
__device__ __forceinline__ double rg_grad(const c128 (&a)[1 << R], const c128 (&b)[1 << R], const DGate &g,
                                          const DDeriv &d, const c128 *__restrict__ mats) {
  constexpr int NR = 1 << R;
  const c128 *__restrict__ D = mats + d.mat;
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
    case GK_DENSE4: v = gr_dense4<NR>(a, b, D); break;
    default: break;
  }
  return v;
}

template <int W>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

template <typename JT>
__device__ __forceinline__ int find_job(const JT *__restrict__ jobs, int n_jobs, int64_t u) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].unit0 <= u) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------ fused LDS pass

template <int K, int R, bool ADJ>
__global__ void __launch_bounds__(1 << (K - R))
k_pass_lds(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units, DOverride ov) {
  constexpr int T = 1 << (K - R);
  constexpr int NR = 1 << R;
  constexpr int WS = T < 64 ? T : 64;
  constexpr int NW = (T + 63) / 64;
  extern __shared__ c128 smem[];
  __shared__ double red[ADJ ? kMaxVarPerPass : 1][NW];
  c128 *la = smem;
  c128 *lb = smem + (1 << K);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;

  for (int64_t u = blockIdx.x; u < total_units; u += gridDim.x) {
    const DJob &J = jobs[find_job(jobs, n_jobs, u)];
    const DPass *__restrict__ P = J.pass;
    const int64_t tile = u - J.unit0;
    c128 *A = ov.use ? ov.a : J.a;
    c128 *Bv = ov.use ? ov.b : J.b;
    const c128 *__restrict__ MT = ov.use ? ov.mats : J.mats;
    double *PT = ov.use ? ov.partials : J.partials;
    const int mode = ov.use ? ov.mode : J.mode;
    uint64_t gbase = (uint64_t)tile;
#pragma unroll
    for (int i = 0; i < K; i++) gbase = ins0<uint64_t>(gbase, P->tq[i]);
    uint64_t st = 0;
#pragma unroll
    for (int i = 0; i < K - R; i++) st |= (uint64_t)((t >> i) & 1) << P->tq[i];
    const c128 *__restrict__ src = A;
    c128 *dst = (mode == 1) ? Bv : A;
    // HBM -> LDS, coalesced over the low tile bits
#pragma unroll
    for (int j = 0; j < NR; j++) {
      uint64_t oj = 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if ((j >> i) & 1) oj |= 1ull << P->tq[K - R + i];
      const uint64_t gi = gbase | st | oj;
      la[swz(j * T + t)] = src[gi];
      if constexpr (ADJ) lb[swz(j * T + t)] = Bv[gi];
    }
    __syncthreads();
    const int nst = P->nst;
    for (int si = 0; si < nst; si++) {
      const int s = ADJ ? nst - 1 - si : si;
      const DStage S = P->stages[s];
      int base = t;
#pragma unroll
      for (int i = 0; i < R; i++) base = ins0<int>(base, S.srt[i]);
      int off[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) {
        int o = 0;
#pragma unroll
        for (int i = 0; i < R; i++)
          if ((j >> i) & 1) o |= 1 << S.rbit[i];
        off[j] = swz(base | o);
      }
      c128 a[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) a[j] = la[off[j]];
      if constexpr (!ADJ) {
        for (int g = S.g0; g < S.g1; g++) rg_apply<R, false>(a, P->gates[g], MT);
      } else {
        c128 b[NR];
#pragma unroll
        for (int j = 0; j < NR; j++) b[j] = lb[off[j]];
        for (int g = S.g1 - 1; g >= S.g0; g--) {
          const DGate G = P->gates[g];
          rg_apply<R, true>(a, G, MT);  // Phi <- Q^dagger Phi
          for (int d = 0; d < G.nd; d++) {  // <Psi| dQ |Phi>
            const DDeriv Dd = P->derivs[G.d0 + d];
            double v = wave_sum<WS>(rg_grad<R>(a, b, G, Dd, MT));
            if (lane == 0) red[Dd.local][wave] = v;
          }
          rg_apply<R, true>(b, G, MT);  // Psi <- Q^dagger Psi
        }
#pragma unroll
        for (int j = 0; j < NR; j++) lb[off[j]] = b[j];
      }
#pragma unroll
      for (int j = 0; j < NR; j++) la[off[j]] = a[j];
      __syncthreads();
    }
    // LDS -> HBM
#pragma unroll
    for (int j = 0; j < NR; j++) {
      uint64_t oj = 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if ((j >> i) & 1) oj |= 1ull << P->tq[K - R + i];
      const uint64_t gi = gbase | st | oj;
      dst[gi] = la[swz(j * T + t)];
      if constexpr (ADJ) Bv[gi] = lb[swz(j * T + t)];
    }
    if constexpr (ADJ) {
      const int nv = P->nvar;
      for (int v = t; v < nv; v += T) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; w++) s += red[v][w];
        PT[(int64_t)P->vslot[v] * J.n_units + tile] = s;
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

template <int R, int MODE>
__global__ void __launch_bounds__(256) k_pass_reg(const DJob *__restrict__ jobs, int n_jobs, int64_t total_units, DOverride ov) {
  constexpr int NR = 1 << R;
  __shared__ double red[MODE ? kMaxVarPerPass : 1][4];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  for (int64_t u = blockIdx.x; u < total_units; u += gridDim.x) {
    const DJob &J = jobs[find_job(jobs, n_jobs, u)];
    const DPass *__restrict__ P = J.pass;
    const int64_t ublk = u - J.unit0;
    c128 *A = ov.use ? ov.a : J.a;
    c128 *Bv = ov.use ? ov.b : J.b;
    const c128 *__restrict__ MT = ov.use ? ov.mats : J.mats;
    double *PT = ov.use ? ov.partials : J.partials;
    const int mode = ov.use ? ov.mode : J.mode;
    const int64_t tiles = (int64_t)1 << (J.nbits - R);
    const int64_t tile = ublk * 256 + t;
    const bool act = tile < tiles;
    const DStage S = P->stages[0];
    uint64_t base = act ? (uint64_t)tile : 0;
#pragma unroll
    for (int i = 0; i < R; i++) base = ins0<uint64_t>(base, P->tq[i]);
    uint64_t off[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) {
      uint64_t o = 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if ((j >> i) & 1) o |= 1ull << P->tq[S.rbit[i]];
      off[j] = base | o;
    }
    c128 a[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) a[j] = act ? A[off[j]] : make_double2(0.0, 0.0);
    if constexpr (MODE == 0) {
      for (int g = S.g0; g < S.g1; g++) rg_apply<R, false>(a, P->gates[g], MT);
      c128 *dst = (mode == 1) ? Bv : A;
      if (act) {
#pragma unroll
        for (int j = 0; j < NR; j++) dst[off[j]] = a[j];
      }
    } else {
      c128 b[NR];
#pragma unroll
      for (int j = 0; j < NR; j++) b[j] = act ? Bv[off[j]] : make_double2(0.0, 0.0);
      for (int g = S.g1 - 1; g >= S.g0; g--) {
        const DGate G = P->gates[g];
        if constexpr (MODE == 1) {
          rg_apply<R, true>(a, G, MT);
          for (int d = 0; d < G.nd; d++) {
            const DDeriv Dd = P->derivs[G.d0 + d];
            const double v = wave_sum<64>(rg_grad<R>(a, b, G, Dd, MT));
            if (lane == 0) red[Dd.local][wave] = v;
          }
        } else {
          if (G.nd > 0) {
            c128 c[NR];
#pragma unroll
            for (int j = 0; j < NR; j++) c[j] = a[j];
            for (int g2 = S.g0; g2 < g; g2++) rg_apply<R, false>(c, P->gates[g2], MT);
            for (int d = 0; d < G.nd; d++) {
              const DDeriv Dd = P->derivs[G.d0 + d];
              const double v = wave_sum<64>(rg_grad<R>(c, b, G, Dd, MT));
              if (lane == 0) red[Dd.local][wave] = v;
            }
          }
        }
        rg_apply<R, true>(b, G, MT);
      }
      if (act) {
#pragma unroll
        for (int j = 0; j < NR; j++) {
          if constexpr (MODE == 1) A[off[j]] = a[j];
          Bv[off[j]] = b[j];
        }
      }
      __syncthreads();
      const int nv = P->nvar;
      for (int v = t; v < nv; v += 256)
        PT[(int64_t)P->vslot[v] * J.n_units + ublk] = (red[v][0] + red[v][1]) + (red[v][2] + red[v][3]);
    }
    __syncthreads();
  }
}


template <int K, int R, bool ADJ>
hipError_t launch_lds_t(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                        hipStream_t st) {
  const size_t shmem = (ADJ ? 2 : 1) * (size_t(1) << K) * sizeof(c128);
  static bool attr_set = false;
  if (!attr_set && shmem > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)k_pass_lds<K, R, ADJ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const int g = grid > 0 ? grid : (int)(total < (1 << 30) ? total : (1 << 30));
  hipLaunchKernelGGL((k_pass_lds<K, R, ADJ>), dim3(g), dim3(1 << (K - R)), shmem, st, jobs, n_jobs, total, ov);
  return hipGetLastError();
}

template <int R, int MODE>
hipError_t launch_reg_t(const DJob *jobs, int n_jobs, int64_t total, int grid, const DOverride &ov,
                        hipStream_t st) {
  const int g = grid > 0 ? grid : (int)(total < (1 << 30) ? total : (1 << 30));
  hipLaunchKernelGGL((k_pass_reg<R, MODE>), dim3(g), dim3(256), 0, st, jobs, n_jobs, total, ov);
  return hipGetLastError();
}

}  // namespace vqc

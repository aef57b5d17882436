/*
 * vqc_oracle.c -- plain, slow, obviously correct CPU oracle for the
 * variational-circuit hot path of "JuliVQC" (Liao et al., arXiv:2406.19212).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the HIP path.
 *
 * Everything is FP64 (double complex) and compiled without FMA contraction.
 * The optional OpenMP loop in or_apply only splits independent outer
 * iterations (the paper's Fig. 4 argument), so results do not depend on the
 * thread count.
 *
 * Conventions (Sec. 2.1):
 *   state index x = sum_k b_k 2^k          qubit k <-> bit k (column-major,
 *                                          first qubit fastest)
 *   mixed state  v[x + 2^n y] = rho[x][y]  ket bits 0..n-1, bra bits n..2n-1
 *   gate matrix  G[r*d + c], d = 2^m       r = output, c = input local index
 *   local index  l = sum_t b_{q_t} 2^t     first listed qubit = LSB
 *
 * Readings of the paper that this file takes (all listed in the design notes):
 *   - Ry = exp(-i theta Y/2) = [[c,-s],[s,c]]; the printed matrix in Sec. 2.2
 *     has -s in both off-diagonal slots, which is not unitary.
 *   - the third printed rotation (labelled Rx) is Rz = diag(e^{-i t/2}, e^{i t/2}).
 *   - depolarizing: K0 = sqrt(1-3p/4) I, K1..3 = sqrt(p/4) sigma (the printed
 *     sqrt(p/2) is not trace preserving); rho -> (1-p) rho + p Tr(rho) I/2.
 *   - two-qubit depolarizing (not in the paper): K0 = sqrt(1-15p/16) I(x)I,
 *     K_ab = sqrt(p/16) sigma_a (x) sigma_b for the 15 non-identity pairs.
 *   - superoperator of Eq. (channel2): S = sum_s conj(K_s) (x) K_s with K_s on
 *     the ket bits (low local bits) and conj(K_s) on the bra bits, i.e.
 *     rho -> sum_s K_s rho K_s^dagger.
 *   - sqrt(G) for G in {X, Y, W}, W = (X+Y)/sqrt(2): the principal root
 *     ((1+i) I + (1-i) G) / 2.
 *   - FSIM local index l = b_{q0} + 2 b_{q1} (column-major tensor order).
 *   - noisy backward: Psi_{j-1} = M_j^dagger Psi_j (adjoint superoperator);
 *     Phi_{j-1} is recomputed from stored states (or_grad_mixed) or, in the
 *     inverse form that Sec. 3.3 says extends Alg. 2 to channels,
 *     Phi_{j-1} = M_j^{-1} Phi_j (or_grad_mixed_inverse).  Using M^{-1} for
 *     Psi as well would give wrong gradients for non-unitary channels.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* oracle-private op codes */
enum {
  OR_X = 1, OR_Y, OR_Z, OR_H, OR_S, OR_T, OR_SX, OR_SY, OR_SW,
  OR_RX, OR_RY, OR_RZ, OR_ID,
  OR_CZ = 20, OR_CNOT, OR_SWAP, OR_ISWAP, OR_FSIM, OR_CRX, OR_CRY, OR_CRZ,
  OR_CONTROL, OR_MATRIX, OR_TOFFOLI, OR_FREDKIN, OR_CCONTROL,
  OR_AD = 40, OR_PD, OR_DEP, OR_DEP2, OR_KRAUS
};

typedef struct {
  int code;
  int m;              /* number of qubits the op acts on */
  int q[4];           /* qubits, 0-based */
  double prm[5];      /* parameter values */
  int var[5];         /* theta index of parameter k, or -1 */
  int n_data;         /* complex entries at data */
  const cplx *data;   /* MATRIX: d*d; CONTROL, CCONTROL: 2*2 target; KRAUS: nk*d*d */
} or_op;

static int is_channel(int code) { return code >= OR_AD; }

/* ------------------------------------------------------------ parameters */

static double param(const or_op *op, const double *theta, int k) {
  if (theta && op->var[k] >= 0) return theta[op->var[k]];
  return op->prm[k];
}

static int n_params_of(int code) {
  switch (code) {
    case OR_RX: case OR_RY: case OR_RZ: case OR_CRX: case OR_CRY: case OR_CRZ: return 1;
    case OR_FSIM: return 5;
    default: return 0;
  }
}

/* --------------------------------------------------------- gate matrices */

/* 2x2 rotation e^{-i t P/2} (Sec. 2.2, with the Ry/Rz readings above) and its
 * derivative w.r.t. t when deriv != 0. */
static void rot1(int code, double t, int deriv, cplx *G) {
  double c = cos(t / 2), s = sin(t / 2);
  if (deriv) {
    /* d/dt cos(t/2) = -s/2, d/dt sin(t/2) = c/2 */
    double dc = -s / 2, ds = c / 2;
    c = dc; s = ds;
  }
  switch (code) {
    case OR_RX: G[0] = c; G[1] = -I * s; G[2] = -I * s; G[3] = c; break;
    case OR_RY: G[0] = c; G[1] = -s; G[2] = s; G[3] = c; break;
    case OR_RZ:
      /* diag(e^{-it/2}, e^{it/2}) and derivative diag(-i/2 e^{-it/2}, i/2 e^{it/2}) */
      if (!deriv) { G[0] = cexp(-I * t / 2); G[3] = cexp(I * t / 2); }
      else { G[0] = -I / 2 * cexp(-I * t / 2); G[3] = I / 2 * cexp(I * t / 2); }
      G[1] = 0; G[2] = 0;
      break;
  }
}

static void zero(cplx *G, int d) { for (int i = 0; i < d * d; i++) G[i] = 0; }

/* CONTROLGate(i, j, U): control = local bit 0, target = local bit 1 */
static void controlled(const cplx *U, int identity_block, cplx *G) {
  zero(G, 4);
  if (identity_block) { G[0 * 4 + 0] = 1; G[2 * 4 + 2] = 1; }
  /* control = 1: local indices 1 (target 0) and 3 (target 1) */
  G[1 * 4 + 1] = U[0]; G[1 * 4 + 3] = U[1];
  G[3 * 4 + 1] = U[2]; G[3 * 4 + 3] = U[3];
}

/* FSIM(theta, phi, D+, D-, Doff) of Sec. 2.2 and its derivatives.
 * k = -1: the matrix; k = 0..4: derivative w.r.t. parameter k. */
static void fsim(const double *p, int k, cplx *G) {
  double th = p[0], ph = p[1], dp = p[2], dm = p[3], doff = p[4];
  cplx e11 = cexp(I * (dp + dm)), e12 = cexp(I * (dp - doff));
  cplx e21 = cexp(I * (dp + doff)), e22 = cexp(I * (dp - dm));
  cplx e33 = cexp(I * (2 * dp - ph));
  cplx c = cos(th), s = sin(th);
  zero(G, 4);
  switch (k) {
    case -1:
      G[0] = 1;
      G[1 * 4 + 1] = e11 * c;        G[1 * 4 + 2] = -I * e12 * s;
      G[2 * 4 + 1] = -I * e21 * s;   G[2 * 4 + 2] = e22 * c;
      G[3 * 4 + 3] = e33;
      break;
    case 0: /* d/dtheta */
      G[1 * 4 + 1] = -e11 * s;       G[1 * 4 + 2] = -I * e12 * c;
      G[2 * 4 + 1] = -I * e21 * c;   G[2 * 4 + 2] = -e22 * s;
      break;
    case 1: /* d/dphi */
      G[3 * 4 + 3] = -I * e33;
      break;
    case 2: /* d/dD+ */
      G[1 * 4 + 1] = I * e11 * c;    G[1 * 4 + 2] = e12 * s;
      G[2 * 4 + 1] = e21 * s;        G[2 * 4 + 2] = I * e22 * c;
      G[3 * 4 + 3] = 2 * I * e33;
      break;
    case 3: /* d/dD- */
      G[1 * 4 + 1] = I * e11 * c;    G[2 * 4 + 2] = -I * e22 * c;
      break;
    case 4: /* d/dDoff */
      G[1 * 4 + 2] = -e12 * s;       G[2 * 4 + 1] = e21 * s;
      break;
  }
}

/* Fill the 2^m x 2^m matrix of a gate op.  Returns its dimension, or -1. */
int or_gate_matrix(const or_op *op, const double *theta, cplx *G) {
  const double r2 = sqrt(0.5);
  cplx U[4];
  switch (op->code) {
    case OR_ID: G[0] = 1; G[1] = 0; G[2] = 0; G[3] = 1; return 2;
    case OR_X: G[0] = 0; G[1] = 1; G[2] = 1; G[3] = 0; return 2;
    case OR_Y: G[0] = 0; G[1] = -I; G[2] = I; G[3] = 0; return 2;
    case OR_Z: G[0] = 1; G[1] = 0; G[2] = 0; G[3] = -1; return 2;
    case OR_H: G[0] = r2; G[1] = r2; G[2] = r2; G[3] = -r2; return 2;
    case OR_S: G[0] = 1; G[1] = 0; G[2] = 0; G[3] = I; return 2;
    case OR_T: G[0] = 1; G[1] = 0; G[2] = 0; G[3] = cexp(I * M_PI / 4); return 2;
    case OR_SX: /* ((1+i) I + (1-i) X) / 2 */
      G[0] = (1 + I) / 2; G[1] = (1 - I) / 2; G[2] = (1 - I) / 2; G[3] = (1 + I) / 2; return 2;
    case OR_SY: /* ((1+i) I + (1-i) Y) / 2 */
      G[0] = (1 + I) / 2; G[1] = -(1 + I) / 2; G[2] = (1 + I) / 2; G[3] = (1 + I) / 2; return 2;
    case OR_SW: /* ((1+i) I + (1-i) W) / 2, W = (X+Y)/sqrt(2) */
      G[0] = (1 + I) / 2; G[1] = -I * r2; G[2] = r2; G[3] = (1 + I) / 2; return 2;
    case OR_RX: case OR_RY: case OR_RZ:
      rot1(op->code, param(op, theta, 0), 0, G); return 2;
    case OR_CZ:
      zero(G, 4); G[0] = 1; G[5] = 1; G[10] = 1; G[15] = -1; return 4;
    case OR_CNOT: /* control q0 (local bit 0), target q1 (local bit 1) */
      zero(G, 4); G[0 * 4 + 0] = 1; G[2 * 4 + 2] = 1; G[3 * 4 + 1] = 1; G[1 * 4 + 3] = 1; return 4;
    case OR_SWAP:
      zero(G, 4); G[0] = 1; G[1 * 4 + 2] = 1; G[2 * 4 + 1] = 1; G[15] = 1; return 4;
    case OR_ISWAP:
      zero(G, 4); G[0] = 1; G[1 * 4 + 2] = I; G[2 * 4 + 1] = I; G[15] = 1; return 4;
    case OR_FSIM: {
      double p[5];
      for (int k = 0; k < 5; k++) p[k] = param(op, theta, k);
      fsim(p, -1, G);
      return 4;
    }
    case OR_CRX: case OR_CRY: case OR_CRZ:
      rot1(op->code - OR_CRX + OR_RX, param(op, theta, 0), 0, U);
      controlled(U, 1, G);
      return 4;
    case OR_CONTROL:
      if (op->n_data != 4) return -1;
      controlled(op->data, 1, G);
      return 4;
    case OR_MATRIX: {
      int d = 1 << op->m;
      if (op->n_data != d * d) return -1;
      for (int i = 0; i < d * d; i++) G[i] = op->data[i];
      return d;
    }
    /* three-qubit gates (Sec. 2.2), local index b_{q0} + 2 b_{q1} + 4 b_{q2} */
    case OR_TOFFOLI: /* controls q0, q1; X on q2 */
      zero(G, 8);
      for (int l = 0; l < 8; l++) G[((l & 3) == 3 ? l ^ 4 : l) * 8 + l] = 1;
      return 8;
    case OR_FREDKIN: /* control q0; swap q1 and q2 */
      zero(G, 8);
      for (int l = 0; l < 8; l++) {
        int o = l;
        if ((l & 1) && ((l >> 1) & 1) != ((l >> 2) & 1)) o = l ^ 6;
        G[o * 8 + l] = 1;
      }
      return 8;
    case OR_CCONTROL: /* controls q0, q1; the 2x2 U on q2 */
      if (op->n_data != 4) return -1;
      zero(G, 8);
      for (int l = 0; l < 8; l++) {
        if ((l & 3) != 3) { G[l * 8 + l] = 1; continue; }
        int b = l >> 2;
        G[l * 8 + (3 | 0)] = op->data[b * 2 + 0];
        G[l * 8 + (3 | 4)] = op->data[b * 2 + 1];
      }
      return 8;
  }
  return -1;
}

/* Derivative of a gate matrix w.r.t. its parameter k. Returns dim or -1. */
int or_gate_dmatrix(const or_op *op, const double *theta, int k, cplx *G) {
  cplx U[4];
  switch (op->code) {
    case OR_RX: case OR_RY: case OR_RZ:
      if (k != 0) return -1;
      rot1(op->code, param(op, theta, 0), 1, G); return 2;
    case OR_CRX: case OR_CRY: case OR_CRZ:
      if (k != 0) return -1;
      rot1(op->code - OR_CRX + OR_RX, param(op, theta, 0), 1, U);
      controlled(U, 0, G);
      return 4;
    case OR_FSIM: {
      double p[5];
      if (k < 0 || k > 4) return -1;
      for (int j = 0; j < 5; j++) p[j] = param(op, theta, j);
      fsim(p, k, G);
      return 4;
    }
  }
  return -1;
}

/* Kraus operators of a channel op (Sec. 2.2).  Returns the count, or -1. */
int or_channel_kraus(const or_op *op, cplx *K) {
  static const cplx pauli[4][4] = {
      {1, 0, 0, 1}, {0, 1, 1, 0}, {0, -I, I, 0}, {1, 0, 0, -1}};
  double g = op->prm[0];
  switch (op->code) {
    case OR_AD:
      K[0] = 1; K[1] = 0; K[2] = 0; K[3] = sqrt(1 - g);
      K[4] = 0; K[5] = sqrt(g); K[6] = 0; K[7] = 0;
      return 2;
    case OR_PD:
      K[0] = 1; K[1] = 0; K[2] = 0; K[3] = sqrt(1 - g);
      K[4] = 0; K[5] = 0; K[6] = 0; K[7] = sqrt(g);
      return 2;
    case OR_DEP:
      for (int s = 0; s < 4; s++) {
        double w = s == 0 ? sqrt(1 - 3 * g / 4) : sqrt(g / 4);
        for (int i = 0; i < 4; i++) K[4 * s + i] = w * pauli[s][i];
      }
      return 4;
    case OR_DEP2:
      /* K_{ab} = w sigma_a (x) sigma_b: sigma_a on local bit 0, sigma_b on bit 1 */
      for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
          int s = a + 4 * b;
          double w = s == 0 ? sqrt(1 - 15 * g / 16) : sqrt(g / 16);
          cplx *M = K + 16 * s;
          for (int r = 0; r < 4; r++)
            for (int c = 0; c < 4; c++)
              M[r * 4 + c] = w * pauli[a][(r & 1) * 2 + (c & 1)] * pauli[b][(r >> 1) * 2 + (c >> 1)];
        }
      return 16;
    case OR_KRAUS: {
      int d = 1 << op->m;
      if (op->n_data <= 0 || op->n_data % (d * d)) return -1;
      for (int i = 0; i < op->n_data; i++) K[i] = op->data[i];
      return op->n_data / (d * d);
    }
  }
  return -1;
}

/* Superoperator of Eq. (channel2), textbook reading:
 * S[(x + d y), (x' + d y')] = sum_s K_s[x][x'] conj(K_s[y][y']). */
void or_superop(int m, int nk, const cplx *K, cplx *S) {
  int d = 1 << m, D = d * d;
  for (int i = 0; i < D * D; i++) S[i] = 0;
  for (int s = 0; s < nk; s++) {
    const cplx *Ks = K + (size_t)s * d * d;
    for (int x = 0; x < d; x++)
      for (int y = 0; y < d; y++)
        for (int x2 = 0; x2 < d; x2++)
          for (int y2 = 0; y2 < d; y2++)
            S[(x + d * y) * D + (x2 + d * y2)] += Ks[x * d + x2] * conj(Ks[y * d + y2]);
  }
}

/* ----------------------------------------------------------- application */

/* Eq. (3) / Eq. (twoqubitgate) / Alg. 1, for m up to 6: for every assignment of
 * the untouched bits, gather the 2^m amplitudes addressed by the op's qubits,
 * multiply by G, scatter back.  The outer loop over untouched bits is the
 * paper's s1, s2, s3 loops merged into one counter t with zero bits inserted
 * at the op's (sorted) positions. */
void or_apply(cplx *v, int nbits, int m, const int *q, const cplx *G) {
  int d = 1 << m;
  int srt[8];
  for (int i = 0; i < m; i++) srt[i] = q[i];
  for (int i = 0; i < m; i++)
    for (int j = i + 1; j < m; j++)
      if (srt[j] < srt[i]) { int t = srt[i]; srt[i] = srt[j]; srt[j] = t; }
  int64_t outer = (int64_t)1 << (nbits - m);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < outer; t++) {
    uint64_t base = (uint64_t)t;
    for (int i = 0; i < m; i++) {
      uint64_t low = base & ((1ull << srt[i]) - 1);
      base = ((base >> srt[i]) << (srt[i] + 1)) | low;
    }
    cplx in[64], out[64];
    uint64_t idx[64];
    for (int l = 0; l < d; l++) {
      uint64_t x = base;
      for (int k = 0; k < m; k++)
        if ((l >> k) & 1) x |= 1ull << q[k];
      idx[l] = x;
      in[l] = v[x];
    }
    for (int r = 0; r < d; r++) {
      cplx acc = 0;
      for (int c = 0; c < d; c++) acc += G[r * d + c] * in[c];
      out[r] = acc;
    }
    for (int l = 0; l < d; l++) v[idx[l]] = out[l];
  }
}

static void dagger(const cplx *G, int d, cplx *Gd) {
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) Gd[c * d + r] = conj(G[r * d + c]);
}

/* superoperator of a unitary gate: S = conj(U) (x) U (one Kraus operator) */
static void gate_superop(const cplx *U, int m, cplx *S) { or_superop(m, 1, U, S); }

/* superoperator derivative: dS = conj(dU) (x) U + conj(U) (x) dU */
static void gate_dsuperop(const cplx *U, const cplx *dU, int m, cplx *S) {
  int d = 1 << m, D = d * d;
  for (int x = 0; x < d; x++)
    for (int y = 0; y < d; y++)
      for (int x2 = 0; x2 < d; x2++)
        for (int y2 = 0; y2 < d; y2++)
          S[(x + d * y) * D + (x2 + d * y2)] =
              dU[x * d + x2] * conj(U[y * d + y2]) + U[x * d + x2] * conj(dU[y * d + y2]);
}

/* the op's superoperator (mixed states): returns the number of local bits */
static int op_superop(const or_op *op, const double *theta, cplx *S) {
  static cplx K[16 * 16 * 16];
  cplx U[256];
  if (is_channel(op->code)) {
    int nk = or_channel_kraus(op, K);
    if (nk < 0) return -1;
    or_superop(op->m, nk, K, S);
  } else {
    if (or_gate_matrix(op, theta, U) < 0) return -1;
    gate_superop(U, op->m, S);
  }
  return 2 * op->m;
}

static void super_qubits(const or_op *op, int n, int *qq) {
  for (int k = 0; k < op->m; k++) { qq[k] = op->q[k]; qq[k + op->m] = op->q[k] + n; }
}

/* Apply one op to a pure (mixed = 0) or vectorised mixed state. */
int or_apply_op(cplx *st, int n, int mixed, const or_op *op, const double *theta) {
  if (op->m < 1 || op->m > 4) return -1;
  for (int k = 0; k < op->m; k++)
    if (op->q[k] < 0 || op->q[k] >= n) return -1;
  if (!mixed) {
    cplx G[256];
    if (is_channel(op->code) || or_gate_matrix(op, theta, G) < 0) return -1;
    or_apply(st, n, op->m, op->q, G);
  } else if (op->m == 3 && is_channel(op->code)) {
    /* three-qubit Kraus set: its 64 x 64 superoperator (Eq. (channel2)) on
     * the ket bits and the bra bits of vec(rho) */
    static cplx K[64 * 64], S[64 * 64];
    int qq[6];
    if (op->code != OR_KRAUS || op->n_data > 64 * 64) return -1;
    int nk = or_channel_kraus(op, K);
    if (nk < 1) return -1;
    or_superop(3, nk, K, S);
    super_qubits(op, n, qq);
    or_apply(st, 2 * n, 6, qq, S);
  } else if (op->m == 3) {
    /* three-qubit gates: rho -> U rho U^dagger as U on the ket bits and
     * conj(U) on the bra bits (the superoperator conj(U) (x) U, applied by
     * factors) */
    cplx G[64], Gc[64];
    int qq[3];
    if (or_gate_matrix(op, theta, G) != 8) return -1;
    for (int i = 0; i < 64; i++) Gc[i] = conj(G[i]);
    for (int k = 0; k < 3; k++) qq[k] = op->q[k] + n;
    or_apply(st, 2 * n, 3, op->q, G);
    or_apply(st, 2 * n, 3, qq, Gc);
  } else {
    cplx S[256];
    int qq[8];
    if (op->m > 2 || op_superop(op, theta, S) < 0) return -1;
    super_qubits(op, n, qq);
    or_apply(st, 2 * n, 2 * op->m, qq, S);
  }
  return 0;
}

/* vec(rho) -> M^dagger vec(rho) = vec(U^dagger rho U) for a three-qubit gate
 * (also its inverse): U^dagger on the ket bits, U^T on the bra bits */
int or_invert(int D, const cplx *A, cplx *Ainv);

/* The 64 x 64 superoperator S of a three-qubit Kraus set (Eq. (channel2)),
 * into a caller buffer of 64 * 64; returns 0 or -1. */
static int kraus3_superop(const or_op *op, cplx *S) {
  cplx *K = malloc(64 * 64 * sizeof(cplx));
  int nk;
  if (!K) return -1;
  if (op->code != OR_KRAUS || op->n_data > 64 * 64 || (nk = or_channel_kraus(op, K)) < 1) {
    free(K);
    return -1;
  }
  or_superop(3, nk, K, S);
  free(K);
  return 0;
}

/* Psi <- S^dagger Psi (adjoint superoperator) or Phi <- S^{-1} Phi (inverse)
 * for a three-qubit channel on vec(rho) of n qubits. */
static int kraus3_apply(cplx *v, int n, const or_op *op, int inverse) {
  cplx *S = malloc(2 * 64 * 64 * sizeof(cplx)), *T = S ? S + 64 * 64 : NULL;
  int qq[8], rc = 0;
  if (!S) return -1;
  if (kraus3_superop(op, S)) rc = -1;
  else if (inverse) rc = or_invert(64, S, T);
  else dagger(S, 64, T);
  if (!rc) {
    super_qubits(op, n, qq);
    or_apply(v, 2 * n, 6, qq, T);
  }
  free(S);
  return rc;
}

static int mixed_gate3_adjoint(cplx *v, int n, const or_op *op, const double *theta) {
  cplx G[64], Gd[64], Gt[64];
  int qq[3];
  if (or_gate_matrix(op, theta, G) != 8) return -1;
  dagger(G, 8, Gd);
  for (int r = 0; r < 8; r++)
    for (int c = 0; c < 8; c++) Gt[r * 8 + c] = G[c * 8 + r];
  for (int k = 0; k < 3; k++) qq[k] = op->q[k] + n;
  or_apply(v, 2 * n, 3, op->q, Gd);
  or_apply(v, 2 * n, 3, qq, Gt);
  return 0;
}

/* Eq. (circuitevolve): run a whole circuit in order. */
int or_run(cplx *st, int n, int mixed, int n_ops, const or_op *ops, const double *theta) {
  for (int j = 0; j < n_ops; j++)
    if (or_apply_op(st, n, mixed, &ops[j], theta)) return -1 - j;
  return 0;
}

/* ----------------------------------------------------------- observables */

static int popc(uint64_t v) { return __builtin_popcountll(v); }

/* phase of P|x> = i^{|Y|} (-1)^{popcount(x & zm)} |x ^ xm> */
static cplx pauli_phase(uint64_t x, uint64_t xm, uint64_t zm) {
  static const cplx ipow[4] = {1, I, -1, -I};
  int k = popc(xm & zm) & 3;
  cplx ph = ipow[k];
  return (popc(x & zm) & 1) ? -ph : ph;
}

/* Sec. 2.5 expectation: pure <psi|H|psi> = sum_t c_t sum_x conj(psi[x^xm]) ph_t(x) psi[x];
 * mixed Tr(H rho) = sum_t c_t sum_y ph_t(y) rho[y][y ^ xm]. */
void or_expect(const cplx *st, int n, int mixed, int nt, const uint64_t *xm,
               const uint64_t *zm, const cplx *coef, cplx *out) {
  uint64_t N = 1ull << n;
  cplx total = 0;
  for (int t = 0; t < nt; t++) {
    cplx acc = 0;
    for (uint64_t x = 0; x < N; x++) {
      if (!mixed)
        acc += conj(st[x ^ xm[t]]) * pauli_phase(x, xm[t], zm[t]) * st[x];
      else
        acc += pauli_phase(x, xm[t], zm[t]) * st[x + N * (x ^ xm[t])];
    }
    total += coef[t] * acc;
  }
  *out = total;
}

/* out = H in, H = sum_t c_t P_t (pure states) */
static void apply_pauli_sum(const cplx *in, int n, int nt, const uint64_t *xm,
                            const uint64_t *zm, const cplx *coef, cplx *out) {
  uint64_t N = 1ull << n;
  for (uint64_t x = 0; x < N; x++) out[x] = 0;
  for (int t = 0; t < nt; t++)
    for (uint64_t x = 0; x < N; x++)
      out[x ^ xm[t]] += coef[t] * pauli_phase(x, xm[t], zm[t]) * in[x];
}

/* vec(H): v[x + 2^n y] = H[x][y] = sum_t c_t <x|P_t|y> */
static void vec_pauli_sum(int n, int nt, const uint64_t *xm, const uint64_t *zm,
                          const cplx *coef, cplx *out) {
  uint64_t N = 1ull << n;
  for (uint64_t i = 0; i < N * N; i++) out[i] = 0;
  for (int t = 0; t < nt; t++)
    for (uint64_t y = 0; y < N; y++)
      out[(y ^ xm[t]) + N * y] += coef[t] * pauli_phase(y, xm[t], zm[t]);
}

static cplx inner(const cplx *a, const cplx *b, uint64_t N) {
  cplx acc = 0;
  for (uint64_t i = 0; i < N; i++) acc += conj(a[i]) * b[i];
  return acc;
}

/* ------------------------------------------------------------- gradients */

/* Sec. 3.3, Alg. 2 (noiseless): L = Re <psi|H|psi>, psi = C init.
 * Phi starts at the final state, Psi = H Phi; walking j = M..1:
 *   Phi <- Q_j^dagger Phi;  g[var] += 2 Re <Psi| dQ_j/dtheta |Phi>;  Psi <- Q_j^dagger Psi.
 * init == NULL means |0..0>.  On return phi_out (if given) holds Phi after the
 * whole sweep, which must equal the initial state. */
int or_grad_pure(int n, int n_ops, const or_op *ops, const double *theta, const cplx *init,
                 int nt, const uint64_t *xm, const uint64_t *zm, const cplx *coef,
                 int n_params, double *grad, double *energy, cplx *phi_out) {
  uint64_t N = 1ull << n;
  cplx *phi = malloc(N * sizeof(cplx)), *psi = malloc(N * sizeof(cplx));
  cplx *tmp = malloc(N * sizeof(cplx));
  cplx G[256], Gd[256], dG[256];
  int rc = 0;
  if (!phi || !psi || !tmp) { rc = -100; goto done; }
  for (uint64_t x = 0; x < N; x++) phi[x] = init ? init[x] : (x == 0);
  if ((rc = or_run(phi, n, 0, n_ops, ops, theta))) goto done;
  apply_pauli_sum(phi, n, nt, xm, zm, coef, psi);
  *energy = creal(inner(phi, psi, N));
  for (int p = 0; p < n_params; p++) grad[p] = 0;
  for (int j = n_ops - 1; j >= 0; j--) {
    const or_op *op = &ops[j];
    int d = or_gate_matrix(op, theta, G);
    if (d < 0) { rc = -1 - j; goto done; }
    dagger(G, d, Gd);
    or_apply(phi, n, op->m, op->q, Gd);
    for (int k = 0; k < n_params_of(op->code); k++) {
      if (op->var[k] < 0) continue;
      if (or_gate_dmatrix(op, theta, k, dG) < 0) { rc = -1 - j; goto done; }
      memcpy(tmp, phi, N * sizeof(cplx));
      or_apply(tmp, n, op->m, op->q, dG);
      grad[op->var[k]] += 2 * creal(inner(psi, tmp, N));
    }
    or_apply(psi, n, op->m, op->q, Gd);
  }
  if (phi_out) memcpy(phi_out, phi, N * sizeof(cplx));
done:
  free(phi); free(psi); free(tmp);
  return rc;
}

/* Sec. 3.5 (noisy): L = <<I| H C |rho0>> = Tr(H rho), rho0 = |0..0><0..0| or init.
 * Psi_M = vec(H); Psi_{j-1} = M_j^dagger Psi_j; for a gate with parameter k,
 * g[var] += Re <<Psi_j| dM_j |Phi_{j-1}>>, dM = conj(dU)(x)U + conj(U)(x)dU,
 * where Phi_{j-1} is the state before op j.  States before op j are
 * recomputed from states stored every `stride` ops (stride <= 0: about
 * sqrt(M)); recomputation repeats the same op sequence, so Phi_{j-1} is
 * bitwise the state of the forward run. */
int or_grad_mixed(int n, int n_ops, const or_op *ops, const double *theta, const cplx *init,
                  int nt, const uint64_t *xm, const uint64_t *zm, const cplx *coef,
                  int n_params, double *grad, double *energy, int stride) {
  uint64_t N = 1ull << (2 * n);
  if (stride <= 0) { stride = 1; while (stride * stride < n_ops) stride++; }
  int n_ck = n_ops / stride + 1;
  cplx **ck = calloc(n_ck, sizeof(cplx *));
  cplx **seg = calloc(stride, sizeof(cplx *));
  cplx *psi = malloc(N * sizeof(cplx)), *tmp = malloc(N * sizeof(cplx));
  cplx *cur = malloc(N * sizeof(cplx));
  cplx S[256], Sd[256], U[256], dU[256], dS[256];
  int qq[8], rc = 0;
  if (!ck || !seg || !psi || !tmp || !cur) { rc = -100; goto done; }
  for (int i = 0; i < n_ck; i++) if (!(ck[i] = malloc(N * sizeof(cplx)))) { rc = -100; goto done; }
  for (int i = 0; i < stride; i++) if (!(seg[i] = malloc(N * sizeof(cplx)))) { rc = -100; goto done; }
  for (uint64_t x = 0; x < N; x++) cur[x] = init ? init[x] : (x == 0);
  /* forward: ck[i] = state before op i*stride */
  for (int j = 0; j < n_ops; j++) {
    if (j % stride == 0) memcpy(ck[j / stride], cur, N * sizeof(cplx));
    if (or_apply_op(cur, n, 1, &ops[j], theta)) { rc = -1 - j; goto done; }
  }
  vec_pauli_sum(n, nt, xm, zm, coef, psi);
  *energy = creal(inner(psi, cur, N));
  for (int p = 0; p < n_params; p++) grad[p] = 0;
  for (int s0 = ((n_ops - 1) / stride) * stride; s0 >= 0; s0 -= stride) {
    int s1 = s0 + stride < n_ops ? s0 + stride : n_ops;
    /* seg[i] = state before op s0 + i */
    memcpy(seg[0], ck[s0 / stride], N * sizeof(cplx));
    for (int j = s0 + 1; j < s1; j++) {
      memcpy(seg[j - s0], seg[j - s0 - 1], N * sizeof(cplx));
      or_apply_op(seg[j - s0], n, 1, &ops[j - 1], theta);
    }
    for (int j = s1 - 1; j >= s0; j--) {
      const or_op *op = &ops[j];
      int D = 1 << (2 * op->m);
      if (op->m == 3) {  /* three-qubit gates and channels carry no parameters */
        if (is_channel(op->code) ? kraus3_apply(psi, n, op, 0) : mixed_gate3_adjoint(psi, n, op, theta)) {
          rc = -1 - j;
          goto done;
        }
        continue;
      }
      super_qubits(op, n, qq);
      if (op_superop(op, theta, S) < 0) { rc = -1 - j; goto done; }
      if (!is_channel(op->code)) {
        or_gate_matrix(op, theta, U);
        for (int k = 0; k < n_params_of(op->code); k++) {
          if (op->var[k] < 0) continue;
          or_gate_dmatrix(op, theta, k, dU);
          gate_dsuperop(U, dU, op->m, dS);
          memcpy(tmp, seg[j - s0], N * sizeof(cplx));
          or_apply(tmp, 2 * n, 2 * op->m, qq, dS);
          grad[op->var[k]] += creal(inner(psi, tmp, N));
        }
      }
      dagger(S, D, Sd);
      or_apply(psi, 2 * n, 2 * op->m, qq, Sd);
    }
  }
done:
  if (ck) for (int i = 0; i < n_ck; i++) free(ck[i]);
  if (seg) for (int i = 0; i < stride; i++) free(seg[i]);
  free(ck); free(seg); free(psi); free(tmp); free(cur);
  return rc;
}

/* Inverse of a D x D row-major matrix (D <= 64) by Gauss-Jordan elimination
 * with partial pivoting (textbook).  Returns 0, or -1 when a pivot is exactly
 * 0. */
int or_invert(int D, const cplx *A, cplx *Ainv) {
  if (D < 1 || D > 64) return -1;
  cplx *W = malloc((size_t)D * 2 * D * sizeof(cplx));
  if (!W) return -1;
  for (int r = 0; r < D; r++)
    for (int c = 0; c < 2 * D; c++) W[r * 2 * D + c] = c < D ? A[r * D + c] : (c - D == r);
  for (int k = 0; k < D; k++) {
    int p = k;
    for (int r = k + 1; r < D; r++)
      if (cabs(W[r * 2 * D + k]) > cabs(W[p * 2 * D + k])) p = r;
    if (W[p * 2 * D + k] == 0) { free(W); return -1; }
    for (int c = 0; c < 2 * D; c++) {
      cplx t = W[k * 2 * D + c];
      W[k * 2 * D + c] = W[p * 2 * D + c];
      W[p * 2 * D + c] = t;
    }
    cplx piv = W[k * 2 * D + k];
    for (int c = 0; c < 2 * D; c++) W[k * 2 * D + c] /= piv;
    for (int r = 0; r < D; r++) {
      if (r == k) continue;
      cplx f = W[r * 2 * D + k];
      for (int c = 0; c < 2 * D; c++) W[r * 2 * D + c] -= f * W[k * 2 * D + c];
    }
  }
  for (int r = 0; r < D; r++)
    for (int c = 0; c < D; c++) Ainv[r * D + c] = W[r * 2 * D + D + c];
  free(W);
  return 0;
}

/* Sec. 3.3 / 3.5, Alg. 2 in the inverse form for noisy circuits: Phi starts
 * at the final vec(rho), Psi = vec(H); walking j = M..1:
 *   Phi <- M_j^{-1} Phi;  g[var] += Re <<Psi| dM_j |Phi>>;  Psi <- M_j^dagger Psi.
 * Only two states are kept.  On return phi_out (if given) holds Phi after the
 * sweep, which equals the initial state up to rounding amplified by the
 * channels' condition numbers.  Returns -1 - j when M_j is singular. */
int or_grad_mixed_inverse(int n, int n_ops, const or_op *ops, const double *theta, const cplx *init,
                          int nt, const uint64_t *xm, const uint64_t *zm, const cplx *coef,
                          int n_params, double *grad, double *energy, cplx *phi_out) {
  uint64_t N = 1ull << (2 * n);
  cplx *phi = malloc(N * sizeof(cplx)), *psi = malloc(N * sizeof(cplx)), *tmp = malloc(N * sizeof(cplx));
  cplx S[256], Si[256], Sd[256], U[256], dU[256], dS[256];
  int qq[8], rc = 0;
  if (!phi || !psi || !tmp) { rc = -100; goto done; }
  for (uint64_t x = 0; x < N; x++) phi[x] = init ? init[x] : (x == 0);
  for (int j = 0; j < n_ops; j++)
    if (or_apply_op(phi, n, 1, &ops[j], theta)) { rc = -1 - j; goto done; }
  vec_pauli_sum(n, nt, xm, zm, coef, psi);
  *energy = creal(inner(psi, phi, N));
  for (int p = 0; p < n_params; p++) grad[p] = 0;
  for (int j = n_ops - 1; j >= 0; j--) {
    const or_op *op = &ops[j];
    int D = 1 << (2 * op->m);
    if (op->m == 3 && is_channel(op->code)) {  /* no parameters: Phi <- S^{-1} Phi, Psi <- S^dagger Psi */
      if (kraus3_apply(phi, n, op, 1) || kraus3_apply(psi, n, op, 0)) {
        rc = -1 - j;
        goto done;
      }
      continue;
    }
    if (op->m == 3) {  /* unitary, no parameters: M^{-1} = M^dagger */
      if (mixed_gate3_adjoint(phi, n, op, theta) || mixed_gate3_adjoint(psi, n, op, theta)) {
        rc = -1 - j;
        goto done;
      }
      continue;
    }
    super_qubits(op, n, qq);
    if (op_superop(op, theta, S) < 0) { rc = -1 - j; goto done; }
    if (or_invert(D, S, Si)) { rc = -1 - j; goto done; }
    or_apply(phi, 2 * n, 2 * op->m, qq, Si);
    if (!is_channel(op->code)) {
      or_gate_matrix(op, theta, U);
      for (int k = 0; k < n_params_of(op->code); k++) {
        if (op->var[k] < 0) continue;
        or_gate_dmatrix(op, theta, k, dU);
        gate_dsuperop(U, dU, op->m, dS);
        memcpy(tmp, phi, N * sizeof(cplx));
        or_apply(tmp, 2 * n, 2 * op->m, qq, dS);
        grad[op->var[k]] += creal(inner(psi, tmp, N));
      }
    }
    dagger(S, D, Sd);
    or_apply(psi, 2 * n, 2 * op->m, qq, Sd);
  }
  if (phi_out) memcpy(phi_out, phi, N * sizeof(cplx));
done:
  free(phi); free(psi); free(tmp);
  return rc;
}

/* ------------------------------------------------- measurement, sampling */

/* weight of basis state x: |psi_x|^2, or rho[x][x] (real part) for vec(rho) */
static double basis_weight(const cplx *st, int n, int mixed, uint64_t x) {
  uint64_t D = 1ull << n;
  if (mixed) return creal(st[x + D * x]);
  return creal(st[x]) * creal(st[x]) + cimag(st[x]) * cimag(st[x]);
}

/* measure!(state, q) of Sec. 2.4: the probability masses s0, s1 of bit q
 * (normalised by their sum), outcome 0 when u < p0 (u uniform in [0,1)
 * supplied by the caller), then the state collapsed onto the outcome and
 * renormalised in place: psi -> P psi / sqrt(s), rho -> P rho P / s.
 * Returns -1 for a state of zero norm. */
int or_measure(cplx *st, int n, int mixed, int q, double u, int *outcome, double *prob) {
  uint64_t D = 1ull << n, len = mixed ? D * D : D;
  double s0 = 0, s1 = 0;
  for (uint64_t x = 0; x < D; x++) {
    double w = basis_weight(st, n, mixed, x);
    if ((x >> q) & 1) s1 += w; else s0 += w;
  }
  double tot = s0 + s1;
  if (!(tot > 0)) return -1;
  int o = u < s0 / tot ? 0 : 1;
  double so = o ? s1 : s0;
  *outcome = o;
  *prob = so / tot;
  double scale = mixed ? 1.0 / so : 1.0 / sqrt(so);
  for (uint64_t i = 0; i < len; i++) {
    int keep = (int)((i >> q) & 1) == o;
    if (mixed) keep = keep && (int)((i >> (q + n)) & 1) == o;
    st[i] = keep ? st[i] * scale : 0;
  }
  return 0;
}

/* Bitstring sampling by the inverse of the cumulative distribution over basis
 * states in index order: sample k is the first x with C(x) > u_k C(D-1),
 * C(x) = sum_{y <= x} weight(y).  Returns -1 for a state of zero norm. */
int or_sample(const cplx *st, int n, int mixed, int count, const double *u, int64_t *out) {
  uint64_t D = 1ull << n;
  double *C = malloc(D * sizeof(double));
  if (!C) return -100;
  double c = 0;
  for (uint64_t x = 0; x < D; x++) { c += basis_weight(st, n, mixed, x); C[x] = c; }
  if (!(c > 0)) { free(C); return -1; }
  for (int k = 0; k < count; k++) {
    double t = u[k] * c;
    uint64_t lo = 0, hi = D - 1;
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (C[mid] > t) hi = mid; else lo = mid + 1;
    }
    out[k] = (int64_t)lo;
  }
  free(C);
  return 0;
}

/* ----------------------------------------------------------------- misc */

void or_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

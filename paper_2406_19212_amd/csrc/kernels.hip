#include "pass_kernels.h"

namespace vqc {

// ------------------------------------------------------ matrices from theta

__device__ __forceinline__ c128 C(double re, double im) { return make_double2(re, im); }

// Gate matrix (k < 0) or derivative w.r.t. parameter k, row-major G[out][in],
// local index b_{q0} + 2 b_{q1}.  Sec. 2.2 definitions: rotations
// exp(-i t P/2) (Ry = [[c,-s],[s,c]], the third rotation is Rz), principal
// square roots ((1+i)I + (1-i)G)/2, CONTROLGate with the control on the first
// qubit, FSIM with (theta, phi, D+, D-, Doff).  Returns the dimension, 0 when
// the derivative is identically zero, -1 on an unknown type.
__device__ int dev_gate(int type, const double *p, int k, const c128 *data, int n_data, c128 *G) {
  const double r2 = 0.70710678118654752440;
  // k == -2: sqrt(X), sqrt(Y), sqrt(W) without their global phase e^{i pi/4}
  if (k == -2) {
    switch (type) {
      case VQC_SX: G[0] = C(r2, 0); G[1] = C(0, -r2); G[2] = C(0, -r2); G[3] = C(r2, 0); return 2;
      case VQC_SY: G[0] = C(r2, 0); G[1] = C(-r2, 0); G[2] = C(r2, 0); G[3] = C(r2, 0); return 2;
      case VQC_SW: G[0] = C(r2, 0); G[1] = C(-0.5, -0.5); G[2] = C(0.5, -0.5); G[3] = C(r2, 0); return 2;
      default: k = -1; break;
    }
  }
  int d = (type >= VQC_CZ) ? 4 : 2;
  if (type == VQC_MATRIX) d = (n_data == 16) ? 4 : 2;
  for (int i = 0; i < d * d; i++) G[i] = C(0, 0);
  if (k >= 0 && !(type == VQC_RX || type == VQC_RY || type == VQC_RZ || type == VQC_CRX || type == VQC_CRY ||
                  type == VQC_CRZ || type == VQC_FSIM))
    return 0;
  switch (type) {
    case VQC_ID: G[0] = C(1, 0); G[3] = C(1, 0); return 2;
    case VQC_X: G[1] = C(1, 0); G[2] = C(1, 0); return 2;
    case VQC_Y: G[1] = C(0, -1); G[2] = C(0, 1); return 2;
    case VQC_Z: G[0] = C(1, 0); G[3] = C(-1, 0); return 2;
    case VQC_H: G[0] = C(r2, 0); G[1] = C(r2, 0); G[2] = C(r2, 0); G[3] = C(-r2, 0); return 2;
    case VQC_S: G[0] = C(1, 0); G[3] = C(0, 1); return 2;
    case VQC_T: G[0] = C(1, 0); G[3] = C(r2, r2); return 2;
    case VQC_SX: G[0] = C(0.5, 0.5); G[1] = C(0.5, -0.5); G[2] = C(0.5, -0.5); G[3] = C(0.5, 0.5); return 2;
    case VQC_SY: G[0] = C(0.5, 0.5); G[1] = C(-0.5, -0.5); G[2] = C(0.5, 0.5); G[3] = C(0.5, 0.5); return 2;
    case VQC_SW: G[0] = C(0.5, 0.5); G[1] = C(0, -r2); G[2] = C(r2, 0); G[3] = C(0.5, 0.5); return 2;
    case VQC_RX: case VQC_RY: case VQC_RZ:
    case VQC_CRX: case VQC_CRY: case VQC_CRZ: {
      double s, c;
      sincos(0.5 * p[0], &s, &c);
      c128 U[4];
      const int base = (type >= VQC_CRX) ? type - VQC_CRX + VQC_RX : type;
      if (k < 0) {
        if (base == VQC_RX) { U[0] = C(c, 0); U[1] = C(0, -s); U[2] = C(0, -s); U[3] = C(c, 0); }
        else if (base == VQC_RY) { U[0] = C(c, 0); U[1] = C(-s, 0); U[2] = C(s, 0); U[3] = C(c, 0); }
        else { U[0] = C(c, -s); U[1] = C(0, 0); U[2] = C(0, 0); U[3] = C(c, s); }
      } else {
        if (base == VQC_RX) { U[0] = C(-0.5 * s, 0); U[1] = C(0, -0.5 * c); U[2] = C(0, -0.5 * c); U[3] = C(-0.5 * s, 0); }
        else if (base == VQC_RY) { U[0] = C(-0.5 * s, 0); U[1] = C(-0.5 * c, 0); U[2] = C(0.5 * c, 0); U[3] = C(-0.5 * s, 0); }
        else { U[0] = C(-0.5 * s, -0.5 * c); U[1] = C(0, 0); U[2] = C(0, 0); U[3] = C(-0.5 * s, 0.5 * c); }
      }
      if (type < VQC_CRX) { for (int i = 0; i < 4; i++) G[i] = U[i]; return 2; }
      if (k < 0) { G[0] = C(1, 0); G[10] = C(1, 0); }
      G[1 * 4 + 1] = U[0]; G[1 * 4 + 3] = U[1]; G[3 * 4 + 1] = U[2]; G[3 * 4 + 3] = U[3];
      return 4;
    }
    case VQC_CZ: G[0] = C(1, 0); G[5] = C(1, 0); G[10] = C(1, 0); G[15] = C(-1, 0); return 4;
    case VQC_CNOT: G[0] = C(1, 0); G[1 * 4 + 3] = C(1, 0); G[2 * 4 + 2] = C(1, 0); G[3 * 4 + 1] = C(1, 0); return 4;
    case VQC_SWAP: G[0] = C(1, 0); G[1 * 4 + 2] = C(1, 0); G[2 * 4 + 1] = C(1, 0); G[15] = C(1, 0); return 4;
    case VQC_ISWAP: G[0] = C(1, 0); G[1 * 4 + 2] = C(0, 1); G[2 * 4 + 1] = C(0, 1); G[15] = C(1, 0); return 4;
    case VQC_FSIM: {
      // entries: (1,1) e^{i(D+ + D-)} cos th, (1,2) -i e^{i(D+ - Doff)} sin th,
      //          (2,1) -i e^{i(D+ + Doff)} sin th, (2,2) e^{i(D+ - D-)} cos th,
      //          (3,3) e^{i(2 D+ - phi)}, (0,0) 1
      const double th = p[0], ph = p[1], dp = p[2], dm = p[3], dof = p[4];
      double st, ct;
      sincos(th, &st, &ct);
      double s11, c11, s12, c12, s21, c21, s22, c22, s33, c33;
      sincos(dp + dm, &s11, &c11);
      sincos(dp - dof, &s12, &c12);
      sincos(dp + dof, &s21, &c21);
      sincos(dp - dm, &s22, &c22);
      sincos(2 * dp - ph, &s33, &c33);
      const c128 e11 = C(c11, s11), e12 = C(c12, s12), e21 = C(c21, s21), e22 = C(c22, s22), e33 = C(c33, s33);
      const c128 mi = C(0, -1), pi_ = C(0, 1);
      // f(th) factors and their derivatives
      double f11 = ct, f12 = st, f22 = ct;
      c128 m11, m12, m21, m22, m33 = C(0, 0), m00 = C(0, 0);
      if (k < 0) {
        m00 = C(1, 0);
        m11 = cscale(f11, e11); m12 = cmul(mi, cscale(f12, e12));
        m21 = cmul(mi, cscale(f12, e21)); m22 = cscale(f22, e22); m33 = e33;
      } else if (k == 0) {
        m11 = cscale(-st, e11); m12 = cmul(mi, cscale(ct, e12));
        m21 = cmul(mi, cscale(ct, e21)); m22 = cscale(-st, e22);
      } else if (k == 1) {
        m11 = m12 = m21 = m22 = C(0, 0);
        m33 = cmul(mi, e33);
      } else if (k == 2) {
        m11 = cmul(pi_, cscale(ct, e11)); m12 = cscale(st, e12);
        m21 = cscale(st, e21); m22 = cmul(pi_, cscale(ct, e22));
        m33 = cmul(C(0, 2), e33);
      } else if (k == 3) {
        m11 = cmul(pi_, cscale(ct, e11)); m12 = m21 = C(0, 0);
        m22 = cmul(mi, cscale(ct, e22));
      } else {
        m11 = m22 = C(0, 0);
        m12 = cscale(-st, e12); m21 = cscale(st, e21);
      }
      G[0] = m00; G[5] = m11; G[6] = m12; G[9] = m21; G[10] = m22; G[15] = m33;
      return 4;
    }
    case VQC_CONTROL:
      G[0] = C(1, 0); G[10] = C(1, 0);
      G[1 * 4 + 1] = data[0]; G[1 * 4 + 3] = data[1]; G[3 * 4 + 1] = data[2]; G[3 * 4 + 3] = data[3];
      return 4;
    case VQC_MATRIX:
      for (int i = 0; i < d * d; i++) G[i] = data[i];
      return d;
  }
  return -1;
}

// Kraus operator s of a channel, element (r, c); Sec. 2.2 channels with the
// trace-preserving depolarizing weights sqrt(1-3p/4), sqrt(p/4) and the
// two-qubit analogue sqrt(1-15p/16), sqrt(p/16) (sigma_a on the first qubit).
__device__ __forceinline__ c128 pauli_el(int a, int r, int c) {
  switch (a) {
    case 0: return C(r == c ? 1.0 : 0.0, 0);
    case 1: return C(r != c ? 1.0 : 0.0, 0);
    case 2: return r == c ? C(0, 0) : (r == 0 ? C(0, -1) : C(0, 1));
    default: return C(r == c ? (r == 0 ? 1.0 : -1.0) : 0.0, 0);
  }
}

__device__ c128 dev_kraus(int type, double g, const c128 *data, int d, int s, int r, int c) {
  switch (type) {
    case VQC_AMPLITUDE_DAMPING:
      if (s == 0) return C(r == c ? (r == 0 ? 1.0 : sqrt(1.0 - g)) : 0.0, 0);
      return C((r == 0 && c == 1) ? sqrt(g) : 0.0, 0);
    case VQC_PHASE_DAMPING:
      if (s == 0) return C(r == c ? (r == 0 ? 1.0 : sqrt(1.0 - g)) : 0.0, 0);
      return C((r == 1 && c == 1) ? sqrt(g) : 0.0, 0);
    case VQC_DEPOLARIZING: {
      const double w = s == 0 ? sqrt(1.0 - 0.75 * g) : sqrt(0.25 * g);
      return cscale(w, pauli_el(s, r, c));
    }
    case VQC_DEPOLARIZING2: {
      const int a = s & 3, b = s >> 2;
      const double w = s == 0 ? sqrt(1.0 - g * (15.0 / 16.0)) : sqrt(g / 16.0);
      return cscale(w, cmul(pauli_el(a, r & 1, c & 1), pauli_el(b, r >> 1, c >> 1)));
    }
    default:  // VQC_KRAUS: row-major blocks
      return data[(s * d + r) * d + c];
  }
}

// rotation i of a shear record from (C, S) = (cos p, sin p)
__device__ __forceinline__ void srec_rot(SRec &r, int i, double C, double S) {
  if (C < 0.0) {
    C = -C;
    S = -S;
    r.neg |= 1u << i;
  }
  r.ab[2 * i] = -S / (1.0 + C);
  r.ab[2 * i + 1] = S;
}

// shear record of a rotation kind from its (row-major) matrix M
__device__ void derive_srec(int kind, const c128 *M, c128 *out) {
  SRec r;
  r.neg = 0;
  r.pad = 0;
  for (int i = 0; i < 7; i++) r.ab[i] = 0.0;
  switch (kind) {
    case GK_SXR1: srec_rot(r, 0, M[0].x, M[2].y); break;  // [[C, -iS], [-iS, C]]: S = Im m10
    case GK_SRR1: srec_rot(r, 0, M[0].x, M[2].x); break;  // [[C, -S], [S, C]]
    case GK_SPH1: srec_rot(r, 0, M[3].x, M[3].y); break;
    case GK_SDG1:
      srec_rot(r, 0, M[0].x, M[0].y);
      srec_rot(r, 1, M[3].x, M[3].y);
      break;
    case GK_SRD1: {
      // m10 = B e^{-i chi}; D^dagger R D is unchanged by chi -> chi + pi,
      // B -> -B, which keeps cos chi >= 0
      double B = hypot(M[2].x, M[2].y), cc = 1.0, sc = 0.0;
      if (B > 0.0) {
        cc = M[2].x / B;
        sc = -M[2].y / B;
      }
      if (cc < 0.0) {
        cc = -cc;
        sc = -sc;
        B = -B;
      }
      srec_rot(r, 0, cc, sc);
      srec_rot(r, 1, M[0].x, B);
      break;
    }
    case GK_SFX:
      srec_rot(r, 0, M[5].x, M[9].y);
      srec_rot(r, 1, M[15].x, M[15].y);
      break;
    default: break;
  }
  *reinterpret_cast<SRec *>(out) = r;  // kSRecSlots c128 slots, 16 B aligned
}

__device__ void build_plain(const DRecipe &R, const c128 *__restrict__ cdata, const double *th, c128 *out);
__device__ void build_fused(const DRecipe &R, const DRecipe *__restrict__ all, const c128 *__restrict__ cdata,
                            const double *th, c128 *out);

__device__ void build_into(const DRecipe &R, const DRecipe *__restrict__ all, const c128 *__restrict__ cdata,
                           const double *th, c128 *out) {
  if (R.form == RF_FUSED || R.form == RF_DFUSED) build_fused(R, all, cdata, th, out);
  else build_plain(R, cdata, th, out);
}

// the recipe's matrix at its output offset, then its shear record
__device__ void build_recipe(const DRecipe &R, const DRecipe *__restrict__ all, const c128 *__restrict__ cdata,
                             const double *th, c128 *out_base) {
  c128 *out = out_base + R.out;
  build_into(R, all, cdata, th, out);
  if (R.shear) {
    const int d = R.nq == 2 ? 4 : 2;
    derive_srec(R.shear, out, out + d * d);
  }
}

// 4x4 superoperator product of a fused run (RF_FUSED / RF_DFUSED)
__device__ void build_fused(const DRecipe &R, const DRecipe *__restrict__ all, const c128 *__restrict__ cdata,
                            const double *th, c128 *out) {
  c128 M[16], S[16], T[16];
  for (int i = 0; i < 16; i++) M[i] = C((i % 5) == 0 ? 1.0 : 0.0, 0.0);
  const int ds = R.form == RF_DFUSED ? R.k >> 3 : -1;
  for (int s = 0; s < R.n_data; s++) {
    DRecipe sub = all[R.data + s];
    if (s == ds) {
      sub.form = RF_DSUPER_GATE;
      sub.k = R.k & 7;
    }
    build_plain(sub, cdata, th, S);
    for (int r = 0; r < 4; r++)
      for (int c = 0; c < 4; c++) {
        c128 acc = C(0, 0);
        for (int k = 0; k < 4; k++) acc = cfma(S[r * 4 + k], M[k * 4 + c], acc);
        T[r * 4 + c] = acc;
      }
    for (int i = 0; i < 16; i++) M[i] = T[i];
  }
  for (int i = 0; i < 16; i++) out[i] = M[i];
}

__device__ void build_plain(const DRecipe &R, const c128 *__restrict__ cdata, const double *th, c128 *out) {
  double p[5];
  for (int k = 0; k < 5; k++) p[k] = (R.pidx[k] >= 0 && th) ? th[R.pidx[k]] : R.pval[k];
  const c128 *data = R.data >= 0 ? cdata + R.data : nullptr;
  c128 G[16], dG[16];
  switch (R.form) {
    case RF_GATE_F: {
      const int d = dev_gate(R.type, p, -2, data, R.n_data, G);
      for (int e = 0; e < d * d; e++) out[e] = G[e];
      break;
    }
    case RF_COPY:
      for (int e = 0; e < R.n_data; e++) out[e] = R.k ? cconj(data[e]) : data[e];
      break;
    case RF_GPHASE: {
      double sn, cs;
      sincospi(0.25 * (R.k & 7), &sn, &cs);
      out[0] = C(cs, sn); out[1] = C(0, 0); out[2] = C(0, 0); out[3] = C(cs, sn);
      break;
    }
    case RF_GATE: case RF_GATE_CONJ: case RF_DGATE: case RF_DGATE_CONJ: {
      int d = dev_gate(R.type, p, (R.form == RF_DGATE || R.form == RF_DGATE_CONJ) ? R.k : -1, data, R.n_data, G);
      if (d <= 0) d = (R.nq == 2) ? 4 : 2;
      const bool cj = (R.form == RF_GATE_CONJ || R.form == RF_DGATE_CONJ);
      for (int e = 0; e < d * d; e++) out[e] = cj ? cconj(G[e]) : G[e];
      break;
    }
    case RF_SUPER_GATE: case RF_DSUPER_GATE: {
      int d = dev_gate(R.type, p, -1, data, R.n_data, G);
      if (R.form == RF_DSUPER_GATE) dev_gate(R.type, p, R.k, data, R.n_data, dG);
      const int D = d * d;
      for (int x = 0; x < d; x++)
        for (int y = 0; y < d; y++)
          for (int x2 = 0; x2 < d; x2++)
            for (int y2 = 0; y2 < d; y2++) {
              c128 v;
              if (R.form == RF_SUPER_GATE) v = cmul(G[x * d + x2], cconj(G[y * d + y2]));
              else v = cadd(cmul(dG[x * d + x2], cconj(G[y * d + y2])), cmul(G[x * d + x2], cconj(dG[y * d + y2])));
              out[(x + d * y) * D + (x2 + d * y2)] = v;
            }
      break;
    }
    case RF_SUPER_KRAUS: {
      const int d = 1 << R.nq, D = d * d;
      if (R.type == VQC_DEPOLARIZING || R.type == VQC_DEPOLARIZING2) {
        // the Pauli Kraus sum in closed form: rho -> (1 - p) rho + p Tr(rho) I / d,
        // S[(x + d y), (x' + d y')] = (1 - p) [x = x'][y = y'] + (p / d) [x = y][x' = y']
        const double g = p[0];
        for (int x = 0; x < d; x++)
          for (int y = 0; y < d; y++)
            for (int x2 = 0; x2 < d; x2++)
              for (int y2 = 0; y2 < d; y2++) {
                double v = (x == x2 && y == y2) ? 1.0 - g : 0.0;
                if (x == y && x2 == y2) v += g / d;
                out[(x + d * y) * D + (x2 + d * y2)] = C(v, 0.0);
              }
        break;
      }
      int nk;
      switch (R.type) {
        case VQC_AMPLITUDE_DAMPING: case VQC_PHASE_DAMPING: nk = 2; break;
        case VQC_DEPOLARIZING: nk = 4; break;
        case VQC_DEPOLARIZING2: nk = 16; break;
        default: nk = R.n_data / (d * d); break;
      }
      for (int x = 0; x < d; x++)
        for (int y = 0; y < d; y++)
          for (int x2 = 0; x2 < d; x2++)
            for (int y2 = 0; y2 < d; y2++) {
              c128 acc = C(0, 0);
              for (int s = 0; s < nk; s++)
                acc = cfma(dev_kraus(R.type, p[0], data, d, s, x, x2), cconj(dev_kraus(R.type, p[0], data, d, s, y, y2)), acc);
              out[(x + d * y) * D + (x2 + d * y2)] = acc;
            }
      break;
    }
    default: break;
  }
}

__global__ void k_build_mats(const DRecipe *__restrict__ rec, int n_rec, const c128 *__restrict__ cdata,
                             const double *const *__restrict__ thetas, c128 *const *__restrict__ mats, int B,
                             const double *theta0, c128 *mats0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n_rec || b >= B) return;
  build_recipe(rec[i], rec, cdata, thetas ? thetas[b] : theta0, mats ? mats[b] : mats0);
}

// op program of a plan for each item: entry i + 1 is op i with its rotation
// record copied from where the recipe built it; entries 0 and n + 1 pad
__global__ void k_assemble(const DGate *__restrict__ gates, const DDeriv *__restrict__ derivs, int n, int prog,
                           c128 *const *__restrict__ mats, int B, c128 *mats0) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n + 2 || b >= B) return;
  c128 *M = mats ? mats[b] : mats0;
  DOp e;
  e.g.kind = GK_NONE;
  e.g.nq = 0;
  for (int t = 0; t < 4; t++) e.g.r[t] = 0;
  e.g.nd = 0;
  e.g.mat = 0;
  e.g.d0 = 0;
  e.neg = 0;
  e.pad = 0;
  for (int k = 0; k < 5; k++) e.ab[k] = 0.0;
  if (i >= 1 && i <= n) {
    e.g = gates[i - 1];
    if (e.g.kind >= GK_SXR1 && e.g.kind <= GK_SFX) {
      const SRec r = *reinterpret_cast<const SRec *>(M + e.g.mat);
      e.neg = r.neg;
      for (int k = 0; k < 4; k++) e.ab[k] = r.ab[k];
    }
    if ((e.g.nd & kGenFlag) && (e.g.nd & 0xff) == 1) {
      const DDeriv d = derivs[e.g.d0];
      e.pad = (1u << 31) | ((uint32_t)(d.local & 0xffff) << 8) | (uint32_t)(d.kind & 0xff);
    }
  }
  *reinterpret_cast<DOp *>(M + prog + (size_t)i * kOpSlots) = e;
}

// Inverse superoperators for the inverse-form noisy adjoint.  Block (i, b)
// inverts item b's D x D matrix at inv[i].mat (D = 4 or 16, any consistent
// storage order) by Gauss-Jordan elimination with partial pivoting in LDS and
// stores the inverse right after it.  kappa_bits receives the largest
// 1-norm condition number ||M|| ||M^{-1}|| as the bits of a non-negative
// double (ordered like the values; inf and NaN from a zero pivot order above
// every finite value).
__global__ void __launch_bounds__(64) k_invert(const DInv *__restrict__ inv, c128 *const *__restrict__ mats,
                                               c128 *mats0, unsigned long long *kappa_bits) {
  __shared__ c128 A[16][33];
  __shared__ c128 f[16];
  __shared__ int piv;
  const int t = threadIdx.x;
  const DInv I = inv[blockIdx.x];
  c128 *M = (mats ? mats[blockIdx.y] : mats0) + I.mat;
  const int D = I.dim, W = 2 * D;
  for (int idx = t; idx < D * W; idx += 64) {
    const int r = idx / W, c = idx % W;
    A[r][c] = c < D ? M[r * D + c] : make_double2(c - D == r ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int k = 0; k < D; k++) {
    if (t == 0) {
      int p = k;
      double best = hypot(A[k][k].x, A[k][k].y);
      for (int r = k + 1; r < D; r++) {
        const double v = hypot(A[r][k].x, A[r][k].y);
        if (v > best) { best = v; p = r; }
      }
      piv = p;
    }
    __syncthreads();
    const int p = piv;
    if (p != k)
      for (int c = t; c < W; c += 64) {
        const c128 x = A[k][c];
        A[k][c] = A[p][c];
        A[p][c] = x;
      }
    __syncthreads();
    const c128 pv = A[k][k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const c128 rp = make_double2(pv.x / den, -pv.y / den);
    __syncthreads();
    for (int c = t; c < W; c += 64) A[k][c] = cmul(A[k][c], rp);
    if (t < D) f[t] = A[t][k];
    __syncthreads();
    for (int idx = t; idx < D * W; idx += 64) {
      const int r = idx / W, c = idx % W;
      if (r != k) A[r][c] = cfma(make_double2(-f[r].x, -f[r].y), A[k][c], A[r][c]);
    }
    __syncthreads();
  }
  for (int idx = t; idx < D * D; idx += 64) M[D * D + idx] = A[idx / D][D + idx % D];
  if (t == 0) {
    double n0 = 0.0, n1 = 0.0;
    bool finite = true;
    for (int c = 0; c < D; c++) {
      double s0 = 0.0, s1 = 0.0;
      for (int r = 0; r < D; r++) {
        s0 += hypot(M[r * D + c].x, M[r * D + c].y);
        s1 += hypot(A[r][D + c].x, A[r][D + c].y);
      }
      finite = finite && (s0 < HUGE_VAL) && (s1 < HUGE_VAL);  // false for inf and NaN
      n0 = fmax(n0, s0);
      n1 = fmax(n1, s1);
    }
    const double kappa = finite ? n0 * n1 : HUGE_VAL;
    atomicMax(kappa_bits, (unsigned long long)__double_as_longlong(kappa));
  }
}

__global__ void k_build_one(DRecipe r, const c128 *__restrict__ cdata, c128 *out) {
  if (threadIdx.x == 0) build_recipe(r, nullptr, cdata, nullptr, out);
}

// -------------------------------------------------- expectation and seeds

constexpr int kEChunk = 4096;  // amplitudes per expectation unit (256 x 16)

__device__ __forceinline__ double2 block_sum2(double2 v, double2 *sh) {
  const int t = threadIdx.x;
  v.x = wave_sum<64>(v.x);
  v.y = wave_sum<64>(v.y);
  if ((t & 63) == 0) sh[t >> 6] = v;
  __syncthreads();
  double2 r = make_double2(0, 0);
  if (t == 0) {
    r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); w++) { r.x += sh[w].x; r.y += sh[w].y; }
  }
  __syncthreads();
  return r;
}

// <psi|H|psi> partial sums (and H psi when J.out != nullptr) for pure states;
// Tr(H rho) partial sums for mixed states (Sec. 2.5).  Term coefficients carry
// i^{|Y|}; the remaining phase is (-1)^{popcount(x & zm)} at the source x.
__global__ void __launch_bounds__(256) k_expect(const DEJob *__restrict__ jobs, int n_jobs, int64_t total_units,
                                                const DTerm *__restrict__ terms, int nt) {
  __shared__ double2 sh[4];
  const int t = threadIdx.x;
  for (int64_t u = blockIdx.x; u < total_units; u += gridDim.x) {
    const DEJob &J = jobs[find_job(jobs, n_jobs, u)];
    const int64_t ublk = u - J.unit0;
    const uint64_t N = 1ull << J.nbits;
    double2 acc = make_double2(0.0, 0.0);
    for (int k = 0; k < kEChunk / 256; k++) {
      const uint64_t y = (uint64_t)ublk * kEChunk + (uint64_t)k * 256 + t;
      if (y >= N) break;
      if (!J.mixed) {
        c128 v = make_double2(0.0, 0.0);
        for (int i = 0; i < nt; i++) {
          const DTerm T = terms[i];
          const uint64_t x = y ^ T.xm;
          c128 c = make_double2(T.cre, T.cim);
          if (__popcll(x & T.zm) & 1) c = make_double2(-c.x, -c.y);
          v = cfma(c, J.psi[x], v);
        }
        const c128 py = J.psi[y];
        acc.x += fma(py.x, v.x, py.y * v.y);
        acc.y += fma(py.x, v.y, -py.y * v.x);
        if (J.out) J.out[y] = v;
      } else {
        for (int i = 0; i < nt; i++) {
          const DTerm T = terms[i];
          c128 c = make_double2(T.cre, T.cim);
          if (__popcll(y & T.zm) & 1) c = make_double2(-c.x, -c.y);
          const c128 r = cmul(c, J.psi[y + N * (y ^ T.xm)]);
          acc.x += r.x;
          acc.y += r.y;
        }
      }
    }
    const double2 s = block_sum2(acc, sh);
    if (t == 0) J.partial[ublk] = s;
  }
}

// vec(H) for the noisy adjoint seed: v[x + 2^n y] = sum_t c_t <x|P_t|y>.
// One lane per column y; terms with equal x-mask accumulate in term order.
__global__ void __launch_bounds__(256) k_seed_mixed(c128 *__restrict__ out, int n, const DTerm *__restrict__ terms,
                                                    int nt) {
  const uint64_t N = 1ull << n;
  for (uint64_t y = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; y < N; y += (uint64_t)gridDim.x * blockDim.x) {
    for (int i = 0; i < nt; i++) {
      const DTerm T = terms[i];
      c128 c = make_double2(T.cre, T.cim);
      if (__popcll(y & T.zm) & 1) c = make_double2(-c.x, -c.y);
      const uint64_t idx = (y ^ T.xm) + N * y;
      out[idx] = cadd(out[idx], c);
    }
  }
}

// second stage: out[j] = sum of job j's partials in a fixed order
__global__ void __launch_bounds__(256) k_reduce_partials(const DEJob *__restrict__ jobs, int n_jobs,
                                                         double2 *__restrict__ out) {
  __shared__ double2 sh[4];
  const int j = blockIdx.x;
  if (j >= n_jobs) return;
  const DEJob &J = jobs[j];
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t i = threadIdx.x; i < J.n_units; i += 256) {
    acc.x += J.partial[i].x;
    acc.y += J.partial[i].y;
  }
  const double2 s = block_sum2(acc, sh);
  if (threadIdx.x == 0) out[j] = s;
}

// real parts into a strided double array (energies)
__global__ void k_take_real(const double2 *__restrict__ in, int n, double *const *__restrict__ dst_ptrs,
                            double *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (dst) dst[i] = in[i].x;
}

// grad[p] = scale * sum over the slots of p (appearance order) of the sum over
// units; one block per (parameter, item), fixed summation order.
__global__ void __launch_bounds__(256) k_grad_reduce(const DGradJob *__restrict__ jobs) {
  __shared__ double2 sh[4];
  const DGradJob &J = jobs[blockIdx.y];
  const int p = blockIdx.x;
  if (p >= J.n_params) return;
  double acc = 0.0;
  for (int k = J.csr_ptr[p]; k < J.csr_ptr[p + 1]; k++) {
    const double *row = J.partials + (int64_t)J.csr_slot[k] * J.n_units;
    for (int64_t i = threadIdx.x; i < J.n_units; i += 256) acc += row[i];
  }
  const double2 s = block_sum2(make_double2(acc, 0.0), sh);
  if (threadIdx.x == 0) J.grad[p] = J.scale * s.x;
}

// ------------------------------------------------------- single-op kernels


// one pair (x, x + 2^q) per lane; PHASE1 touches only the |1> half
__global__ void __launch_bounds__(256) k_g1(c128 *__restrict__ psi, int nbits, int q, const c128 *__restrict__ M,
                                            int kind) {
  const uint64_t half = 1ull << (nbits - 1);
  const c128 m00 = M[0], m01 = M[1], m10 = M[2], m11 = M[3];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < half; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x0 = ins0<uint64_t>(i, q), x1 = x0 | (1ull << q);
    if (kind == SK_PHASE1) {
      psi[x1] = cmul(m11, psi[x1]);
    } else if (kind == SK_DIAG1) {
      psi[x0] = cmul(m00, psi[x0]);
      psi[x1] = cmul(m11, psi[x1]);
    } else {
      const c128 a = psi[x0], b = psi[x1];
      psi[x0] = cfma(m00, a, cmul(m01, b));
      psi[x1] = cfma(m10, a, cmul(m11, b));
    }
  }
}

// one quad per lane (q0 -> local bit 0, q1 -> local bit 1); structured kinds
// read and write only the amplitudes that change
__global__ void __launch_bounds__(256) k_g2(c128 *__restrict__ psi, int nbits, int q0, int q1,
                                            const c128 *__restrict__ M, int kind) {
  const uint64_t quarter = 1ull << (nbits - 2);
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < quarter;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x0 = ins0<uint64_t>(ins0<uint64_t>(i, lo), hi);
    const uint64_t x1 = x0 | (1ull << q0), x2 = x0 | (1ull << q1), x3 = x1 | x2;
    switch (kind) {
      case SK_PHASE11: psi[x3] = cmul(M[15], psi[x3]); break;
      case SK_DIAG2:
        psi[x0] = cmul(M[0], psi[x0]); psi[x1] = cmul(M[5], psi[x1]);
        psi[x2] = cmul(M[10], psi[x2]); psi[x3] = cmul(M[15], psi[x3]);
        break;
      case SK_CX: { const c128 a = psi[x1]; psi[x1] = psi[x3]; psi[x3] = a; break; }
      case SK_CTRL: {
        const c128 a = psi[x1], b = psi[x3];
        psi[x1] = cfma(M[5], a, cmul(M[7], b));
        psi[x3] = cfma(M[13], a, cmul(M[15], b));
        break;
      }
      case SK_FSIM: {
        const c128 a = psi[x1], b = psi[x2];
        psi[x1] = cfma(M[5], a, cmul(M[6], b));
        psi[x2] = cfma(M[9], a, cmul(M[10], b));
        psi[x3] = cmul(M[15], psi[x3]);
        break;
      }
      default: {
        const c128 v0 = psi[x0], v1 = psi[x1], v2 = psi[x2], v3 = psi[x3];
        c128 o[4];
        for (int r = 0; r < 4; r++)
          o[r] = cfma(M[r * 4 + 3], v3, cfma(M[r * 4 + 2], v2, cfma(M[r * 4 + 1], v1, cmul(M[r * 4], v0))));
        psi[x0] = o[0]; psi[x1] = o[1]; psi[x2] = o[2]; psi[x3] = o[3];
      }
    }
  }
}

// generic dense 2^m x 2^m op (m = 3, 4): superoperators of 2q channels
template <int m>
__global__ void __launch_bounds__(256) k_gm(c128 *__restrict__ psi, int nbits, int4 q, const c128 *__restrict__ M) {
  constexpr int d = 1 << m;
  int qs[4] = {q.x, q.y, q.z, q.w}, srt[4];
  for (int i = 0; i < m; i++) srt[i] = qs[i];
  for (int i = 0; i < m; i++)
    for (int j = i + 1; j < m; j++)
      if (srt[j] < srt[i]) { const int tmp = srt[i]; srt[i] = srt[j]; srt[j] = tmp; }
  const uint64_t groups = 1ull << (nbits - m);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < groups;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t base = i;
    for (int k = 0; k < m; k++) base = ins0<uint64_t>(base, srt[k]);
    c128 x[d];
    uint64_t idx[d];
#pragma unroll
    for (int l = 0; l < d; l++) {
      uint64_t o = base;
#pragma unroll
      for (int k = 0; k < m; k++)
        if ((l >> k) & 1) o |= 1ull << qs[k];
      idx[l] = o;
      x[l] = psi[o];
    }
#pragma unroll
    for (int r = 0; r < d; r++) {
      c128 acc = cmul(M[r * d], x[0]);
#pragma unroll
      for (int c = 1; c < d; c++) acc = cfma(M[r * d + c], x[c], acc);
      psi[idx[r]] = acc;
    }
  }
}

// three-qubit channel on vec(rho), Eq. (channel2), on the 8 x 8 blocks of rho
// with ket bits qk (x, y, z: local bits 0, 1, 2) and bra bits qb (physical
// positions; qb = qk + n in the standard layout).  One wave per block: lane
// a + 8 b holds rho[a][b]; the block goes through LDS and each lane forms its
// own entry of
//   dense = 0: sum_s K_s rho K_s^dagger (the Kraus sum term by term,
//              sum_{c,d} K_s[a][c] rho[c][d] conj(K_s[b][d]); K: nk row-major
//              8 x 8 matrices)
//   dense = 1: sum_{l'} S[a + 8 b][l'] v_{l'}, S a row-major 64 x 64
//              superoperator in the same index order (used for the inverse
//              of a channel's superoperator)
// The loop trip count is block-uniform (waves past the last block idle
// through the barriers).
__global__ void __launch_bounds__(256) k_kraus3(c128 *__restrict__ v, int nbits, int4 qk, int4 qb,
                                                const c128 *__restrict__ K, int nk, int dense) {
  __shared__ c128 xs[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a = lane & 7, b = lane >> 3;
  const int pos[6] = {qk.x, qk.y, qk.z, qb.x, qb.y, qb.z};
  int srt[6];
  for (int i = 0; i < 6; i++) srt[i] = pos[i];
  for (int i = 0; i < 6; i++)
    for (int j = i + 1; j < 6; j++)
      if (srt[j] < srt[i]) { const int tmp = srt[i]; srt[i] = srt[j]; srt[j] = tmp; }
  uint64_t off = 0;
  for (int k = 0; k < 3; k++) {
    if ((a >> k) & 1) off |= 1ull << pos[k];
    if ((b >> k) & 1) off |= 1ull << pos[3 + k];
  }
  const uint64_t blocks = 1ull << (nbits - 6);
  for (uint64_t g0 = (uint64_t)blockIdx.x * 4; g0 < blocks; g0 += (uint64_t)gridDim.x * 4) {
    const uint64_t g = g0 + w;
    const bool ok = g < blocks;
    uint64_t base = g;
    for (int k = 0; k < 6; k++) base = ins0<uint64_t>(base, srt[k]);
    if (ok) xs[w][lane] = v[base | off];
    __syncthreads();
    c128 y = make_double2(0.0, 0.0);
    if (ok && dense) {
      const c128 *Sr = K + 64 * lane;
      for (int l = 0; l < 64; l++) y = cfma(Sr[l], xs[w][l], y);
    } else if (ok) {
      for (int s = 0; s < nk; s++) {
        const c128 *Ks = K + 64 * s;
        for (int c = 0; c < 8; c++) {
          c128 t = make_double2(0.0, 0.0);
          for (int d = 0; d < 8; d++) t = cfma(xs[w][c + 8 * d], cconj(Ks[8 * b + d]), t);
          y = cfma(Ks[8 * a + c], t, y);
        }
      }
    }
    __syncthreads();  // every lane has read the block before the next one is staged
    if (ok) v[base | off] = y;
  }
}

// ------------------------------------------------------------------ misc

__global__ void k_init_basis0(c128 *__restrict__ v, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
}

__global__ void k_init_batched(c128 *const *__restrict__ ptrs, const uint64_t *__restrict__ sizes) {
  c128 *v = ptrs[blockIdx.y];
  const uint64_t N = sizes[blockIdx.y];
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = make_double2(i == 0 ? 1.0 : 0.0, 0.0);
}

__global__ void k_fill_u32(uint32_t *__restrict__ v, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = 0u;
}

__global__ void k_fill_zero(c128 *__restrict__ v, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = make_double2(0.0, 0.0);
}

__global__ void k_copy(c128 *__restrict__ dst, const c128 *__restrict__ src, uint64_t N) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// ------------------------------------------------ measurement and sampling

constexpr int kPChunk = 4096;  // basis states per probability block (256 lanes x 16)

// probability weight of basis state x: |psi_x|^2, or rho[x][x] on vec(rho)
__device__ __forceinline__ double basis_weight(const c128 *__restrict__ v, uint64_t x, int n, int mixed) {
  if (mixed) return v[x * ((1ull << n) + 1)].x;
  const c128 a = v[x];
  return fma(a.x, a.x, a.y * a.y);
}

// measure! (Sec. 2.4): per block of kPChunk basis states, the probability
// mass with bit q clear (.x) and set (.y), in a fixed summation order
__global__ void __launch_bounds__(256) k_bit_mass(const c128 *__restrict__ v, int n, int mixed, int q,
                                                  double2 *__restrict__ part) {
  __shared__ double2 sh[4];
  const uint64_t D = 1ull << n, base = (uint64_t)blockIdx.x * kPChunk;
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < kPChunk / 256; k++) {
    const uint64_t x = base + (uint64_t)k * 256 + threadIdx.x;
    if (x < D) {
      const double w = basis_weight(v, x, n, mixed);
      if ((x >> q) & 1) acc.y += w;
      else acc.x += w;
    }
  }
  const double2 r = block_sum2(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// out[0] = sum of m pairs in a fixed order (one block)
__global__ void __launch_bounds__(256) k_sum2(const double2 *__restrict__ in, int64_t m, double2 *__restrict__ out) {
  __shared__ double2 sh[4];
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    acc.x += in[i].x;
    acc.y += in[i].y;
  }
  const double2 r = block_sum2(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}

// collapse onto bit q = outcome: psi -> P psi * scale (scale = 1/sqrt(p)),
// vec(rho) -> (P (x) P) vec(rho) * scale (scale = 1/p)
__global__ void __launch_bounds__(256) k_collapse(c128 *__restrict__ v, uint64_t len, int n, int mixed, int q,
                                                  int outcome, double scale) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (uint64_t)gridDim.x * 256) {
    bool keep = (int)((i >> q) & 1) == outcome;
    if (mixed) keep = keep && (int)((i >> (q + n)) & 1) == outcome;
    const c128 a = v[i];
    v[i] = keep ? make_double2(a.x * scale, a.y * scale) : make_double2(0.0, 0.0);
  }
}

// sampling, step 1: the probability mass of each block of kPChunk basis states
__global__ void __launch_bounds__(256) k_chunk_mass(const c128 *__restrict__ v, int n, int mixed,
                                                    double *__restrict__ mass) {
  __shared__ double2 sh[4];
  const uint64_t D = 1ull << n, base = (uint64_t)blockIdx.x * kPChunk;
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < kPChunk / 256; k++) {
    const uint64_t x = base + (uint64_t)k * 256 + threadIdx.x;
    if (x < D) acc.x += basis_weight(v, x, n, mixed);
  }
  const double2 r = block_sum2(acc, sh);
  if (threadIdx.x == 0) mass[blockIdx.x] = r.x;
}

// step 2: inclusive prefix of the m chunk masses (one block: each thread sums
// a contiguous segment, thread 0 scans the segment sums, each thread then
// writes its segment's running sums)
__global__ void __launch_bounds__(256) k_prefix(const double *__restrict__ mass, int64_t m, double *__restrict__ pref) {
  __shared__ double seg[256];
  const int t = threadIdx.x;
  const int64_t per = (m + 255) / 256, i0 = t * per, i1 = i0 + per < m ? i0 + per : m;
  double s = 0.0;
  for (int64_t i = i0; i < i1; i++) s += mass[i];
  seg[t] = s;
  __syncthreads();
  if (t == 0) {
    double c = 0.0;
    for (int k = 0; k < 256; k++) {
      const double x = seg[k];
      seg[k] = c;
      c += x;
    }
  }
  __syncthreads();
  double c = seg[t];
  for (int64_t i = i0; i < i1; i++) {
    c += mass[i];
    pref[i] = c;
  }
}

// step 3: per sample, the first chunk whose running mass exceeds u * total
// and the mass r still to cover inside it; samples are counted per chunk
__global__ void __launch_bounds__(256) k_locate(const double *__restrict__ pref, int64_t m,
                                                const double *__restrict__ u, int count, int32_t *__restrict__ chunk,
                                                double *__restrict__ rem, uint32_t *__restrict__ cnt) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= count) return;
  const double target = u[k] * pref[m - 1];
  int64_t lo = 0, hi = m - 1;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (pref[mid] > target) hi = mid;
    else lo = mid + 1;
  }
  chunk[k] = (int32_t)lo;
  rem[k] = target - (lo > 0 ? pref[lo - 1] : 0.0);
  atomicAdd(&cnt[lo], 1u);
}

// step 4: exclusive prefix of the per-chunk counts (one block, as k_prefix)
__global__ void __launch_bounds__(256) k_count_offsets(const uint32_t *__restrict__ cnt, int64_t m,
                                                       uint32_t *__restrict__ off) {
  __shared__ uint32_t seg[256];
  const int t = threadIdx.x;
  const int64_t per = (m + 255) / 256, i0 = t * per, i1 = i0 + per < m ? i0 + per : m;
  uint32_t s = 0;
  for (int64_t i = i0; i < i1; i++) s += cnt[i];
  seg[t] = s;
  __syncthreads();
  if (t == 0) {
    uint32_t c = 0;
    for (int k = 0; k < 256; k++) {
      const uint32_t x = seg[k];
      seg[k] = c;
      c += x;
    }
  }
  __syncthreads();
  uint32_t c = seg[t];
  for (int64_t i = i0; i < i1; i++) {
    off[i] = c;
    c += cnt[i];
  }
}

// step 5: sample indices grouped by chunk
__global__ void __launch_bounds__(256) k_bucket(const int32_t *__restrict__ chunk, int count,
                                                const uint32_t *__restrict__ off, uint32_t *__restrict__ cursor,
                                                int32_t *__restrict__ perm) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= count) return;
  const int32_t b = chunk[k];
  perm[off[b] + atomicAdd(&cursor[b], 1u)] = k;
}

// step 6: one block per chunk that holds samples.  The chunk's kPChunk
// weights are read once into LDS with their running sums (16 consecutive
// weights per thread, then the threads' offsets); each of the chunk's samples
// takes the first basis state whose running sum exceeds its r.  Rounding can
// leave r past the chunk's last running sum; the sample is then the chunk's
// last basis state of nonzero weight.
__global__ void __launch_bounds__(256) k_resolve(const c128 *__restrict__ v, int n, int mixed,
                                                 const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ off,
                                                 const int32_t *__restrict__ perm, const double *__restrict__ rem,
                                                 int64_t *__restrict__ out) {
  __shared__ double P[kPChunk];
  __shared__ double seg[256];
  __shared__ int last_nz;
  const int b = blockIdx.x, t = threadIdx.x;
  const uint32_t nb = cnt[b];
  if (nb == 0) return;  // the whole block leaves together
  const uint64_t D = 1ull << n, base = (uint64_t)b * kPChunk;
  double w[16];
  double s = 0.0;
  int my_last = -1;
  for (int k = 0; k < 16; k++) {
    const uint64_t x = base + (uint64_t)t * 16 + k;
    w[k] = x < D ? basis_weight(v, x, n, mixed) : 0.0;
    s += w[k];
    if (w[k] > 0.0) my_last = t * 16 + k;
  }
  seg[t] = s;
  if (t == 0) last_nz = -1;
  __syncthreads();
  atomicMax(&last_nz, my_last);
  if (t == 0) {
    double c = 0.0;
    for (int k = 0; k < 256; k++) {
      const double x = seg[k];
      seg[k] = c;
      c += x;
    }
  }
  __syncthreads();
  double c = seg[t];
  for (int k = 0; k < 16; k++) {
    c += w[k];
    P[t * 16 + k] = c;
  }
  __syncthreads();
  for (uint32_t j = t; j < nb; j += 256) {
    const int32_t k = perm[off[b] + j];
    const double r = rem[k];
    int lo = 0, hi = kPChunk - 1;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (P[mid] > r) hi = mid;
      else lo = mid + 1;
    }
    const int pick = (P[lo] > r || last_nz < 0) ? lo : last_nz;
    out[k] = (int64_t)(base + (uint64_t)pick);
  }
}

__global__ void k_gather(const c128 *__restrict__ psi, const int64_t *__restrict__ idx, int count,
                         c128 *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = psi[idx[i]];
}

struct Mat16 { c128 m[16]; };

__global__ void k_set_mat(c128 *__restrict__ dst, Mat16 m, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = m.m[i];
}

// ------------------------------------------------------------- launchers

static int grid_for(uint64_t work, int block) {
  uint64_t g = (work + block - 1) / block;
  const uint64_t cap = 256ull * 64;  // 256 CUs x 64 blocks: enough in flight
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

// per-instantiation launchers live in inst_*.hip (compiled in parallel)
#define VQC_DECL_LDS(KK, RR, AA) \
  hipError_t launch_lds_##KK##_##RR##_##AA(const DJob *, int, int64_t, int, const DOverride &, hipStream_t);
#define VQC_DECL_REG(RR, MM) \
  hipError_t launch_reg_##RR##_##MM(const DJob *, int, int64_t, int, const DOverride &, hipStream_t);
#include "inst_list.h"
#undef VQC_DECL_LDS
#undef VQC_DECL_REG

hipError_t launch_pass_lds(int K, int R, bool adj, bool d4, const DJob *jobs, int n_jobs, int64_t total, int grid,
                           const DOverride &ov, hipStream_t st) {
  const int mode = (adj ? 1 : 0) | (d4 ? 2 : 0);
#define VQC_DECL_LDS(KK, RR, AA) \
  if (K == KK && R == RR && mode == AA) return launch_lds_##KK##_##RR##_##AA(jobs, n_jobs, total, grid, ov, st);
#define VQC_DECL_REG(RR, MM)
#include "inst_list.h"
#undef VQC_DECL_LDS
#undef VQC_DECL_REG
  return hipErrorInvalidValue;
}

hipError_t launch_pass_reg(int R, int mode, const DJob *jobs, int n_jobs, int64_t total, int grid,
                           const DOverride &ov, hipStream_t st) {
#define VQC_DECL_LDS(KK, RR, AA)
#define VQC_DECL_REG(RR, MM) \
  if (R == RR && mode == MM) return launch_reg_##RR##_##MM(jobs, n_jobs, total, grid, ov, st);
#include "inst_list.h"
#undef VQC_DECL_LDS
#undef VQC_DECL_REG
  return hipErrorInvalidValue;
}

hipError_t launch_build_mats(const DRecipe *rec, int n_rec, const c128 *cdata, const double *const *thetas,
                             c128 *const *mats, int B, const double *theta0, c128 *mats0, hipStream_t st) {
  if (n_rec == 0 || B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_mats, dim3((n_rec + 63) / 64, B), dim3(64), 0, st, rec, n_rec, cdata, thetas, mats, B,
                     theta0, mats0);
  return hipGetLastError();
}

int64_t expect_units(int nbits_iter) {
  const int64_t N = int64_t(1) << nbits_iter;
  return (N + kEChunk - 1) / kEChunk;
}

hipError_t launch_expect(const DEJob *jobs, int n_jobs, int64_t total, const DTerm *terms, int nt, hipStream_t st) {
  const int g = (int)(total < 256 * 32 ? total : 256 * 32);
  hipLaunchKernelGGL(k_expect, dim3(g), dim3(256), 0, st, jobs, n_jobs, total, terms, nt);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const DEJob *jobs, int n_jobs, double2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(n_jobs), dim3(256), 0, st, jobs, n_jobs, out);
  return hipGetLastError();
}

hipError_t launch_take_real(const double2 *in, int n, double *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_take_real, dim3((n + 255) / 256), dim3(256), 0, st, in, n, nullptr, dst);
  return hipGetLastError();
}

hipError_t launch_seed_mixed(c128 *out, int n, const DTerm *terms, int nt, hipStream_t st) {
  const uint64_t N = 1ull << n;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(N * N, 256)), dim3(256), 0, st, out, N * N);
  hipLaunchKernelGGL(k_seed_mixed, dim3(grid_for(N, 256)), dim3(256), 0, st, out, n, terms, nt);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const DGradJob *jobs, int n_items, int max_params, hipStream_t st) {
  if (max_params <= 0 || n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_reduce, dim3(max_params, n_items), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_g1(c128 *psi, int nbits, int q, const c128 *M, int kind, hipStream_t st) {
  hipLaunchKernelGGL(k_g1, dim3(grid_for(1ull << (nbits - 1), 256)), dim3(256), 0, st, psi, nbits, q, M, kind);
  return hipGetLastError();
}

hipError_t launch_g2(c128 *psi, int nbits, int q0, int q1, const c128 *M, int kind, hipStream_t st) {
  hipLaunchKernelGGL(k_g2, dim3(grid_for(1ull << (nbits - 2), 256)), dim3(256), 0, st, psi, nbits, q0, q1, M, kind);
  return hipGetLastError();
}

hipError_t launch_gm(c128 *psi, int nbits, int m, const int *q, const c128 *M, hipStream_t st) {
  const int4 qq = make_int4(q[0], q[1], m > 2 ? q[2] : 0, m > 3 ? q[3] : 0);
  const dim3 grid(grid_for(1ull << (nbits - m), 256));
  if (m == 3) hipLaunchKernelGGL(k_gm<3>, grid, dim3(256), 0, st, psi, nbits, qq, M);
  else if (m == 4) hipLaunchKernelGGL(k_gm<4>, grid, dim3(256), 0, st, psi, nbits, qq, M);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_kraus3(c128 *v, int nbits, int n, const int *q, const c128 *K, int nk, hipStream_t st) {
  const int qb[3] = {q[0] + n, q[1] + n, q[2] + n};
  return launch_block6(v, nbits, q, qb, K, nk, 0, st);
}

hipError_t launch_block6(c128 *v, int nbits, const int *qk, const int *qb, const c128 *K, int nk, int dense,
                         hipStream_t st) {
  if (nbits < 6 || (!dense && nk < 1)) return hipErrorInvalidValue;
  const int4 k4 = make_int4(qk[0], qk[1], qk[2], 0), b4 = make_int4(qb[0], qb[1], qb[2], 0);
  const dim3 grid(grid_for(1ull << (nbits - 6), 4));
  hipLaunchKernelGGL(k_kraus3, grid, dim3(256), 0, st, v, nbits, k4, b4, K, nk, dense);
  return hipGetLastError();
}

hipError_t launch_init_basis0(c128 *v, uint64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_init_basis0, dim3(grid_for(N, 256)), dim3(256), 0, st, v, N);
  return hipGetLastError();
}

hipError_t launch_assemble(const DGate *gates, const DDeriv *derivs, int n_gates, int prog, c128 *const *mats,
                           int B, c128 *mats0, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_assemble, dim3((n_gates + 2 + 63) / 64, B), dim3(64), 0, st, gates, derivs, n_gates, prog,
                     mats, B, mats0);
  return hipGetLastError();
}

hipError_t launch_invert(const DInv *inv, int n_inv, c128 *const *mats, int B, c128 *mats0,
                         unsigned long long *kappa_bits, hipStream_t st) {
  if (n_inv <= 0 || B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_invert, dim3(n_inv, B), dim3(64), 0, st, inv, mats, mats0, kappa_bits);
  return hipGetLastError();
}

hipError_t launch_build_one(const DRecipe &r, const c128 *cdata, c128 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_build_one, dim3(1), dim3(64), 0, st, r, cdata, out);
  return hipGetLastError();
}

hipError_t launch_init_batched(c128 *const *ptrs, const uint64_t *sizes, int B, uint64_t max_n, hipStream_t st) {
  hipLaunchKernelGGL(k_init_batched, dim3(grid_for(max_n, 256) / B + 1, B), dim3(256), 0, st, ptrs, sizes);
  return hipGetLastError();
}

hipError_t launch_fill_zero(c128 *v, uint64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(N, 256)), dim3(256), 0, st, v, N);
  return hipGetLastError();
}

hipError_t launch_copy(c128 *dst, const c128 *src, uint64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(N, 256)), dim3(256), 0, st, dst, src, N);
  return hipGetLastError();
}

int64_t prob_chunks(int n) { return ((int64_t(1) << n) + kPChunk - 1) / kPChunk; }

hipError_t launch_bit_mass(const c128 *v, int n, int mixed, int q, double2 *part, double2 *out, hipStream_t st) {
  const int64_t m = prob_chunks(n);
  hipLaunchKernelGGL(k_bit_mass, dim3((unsigned)m), dim3(256), 0, st, v, n, mixed, q, part);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(256), 0, st, part, m, out);
  return hipGetLastError();
}

hipError_t launch_collapse(c128 *v, uint64_t len, int n, int mixed, int q, int outcome, double scale,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_collapse, dim3(grid_for(len, 256)), dim3(256), 0, st, v, len, n, mixed, q, outcome, scale);
  return hipGetLastError();
}

hipError_t launch_sample(const c128 *v, int n, int mixed, const SampleBufs &sb, const double *u, int count,
                         int64_t *out, hipStream_t st) {
  const int64_t m = prob_chunks(n);
  hipLaunchKernelGGL(k_chunk_mass, dim3((unsigned)m), dim3(256), 0, st, v, n, mixed, sb.mass);
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(256), 0, st, sb.mass, m, sb.pref);
  if (count <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(2 * m, 256)), dim3(256), 0, st, sb.cnt, (uint64_t)(2 * m));
  const unsigned gs = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(k_locate, dim3(gs), dim3(256), 0, st, sb.pref, m, u, count, sb.chunk, sb.rem, sb.cnt);
  hipLaunchKernelGGL(k_count_offsets, dim3(1), dim3(256), 0, st, sb.cnt, m, sb.off);
  hipLaunchKernelGGL(k_bucket, dim3(gs), dim3(256), 0, st, sb.chunk, count, sb.off, sb.cnt + m, sb.perm);
  hipLaunchKernelGGL(k_resolve, dim3((unsigned)m), dim3(256), 0, st, v, n, mixed, sb.cnt, sb.off, sb.perm, sb.rem,
                     out);
  return hipGetLastError();
}

hipError_t launch_gather(const c128 *psi, const int64_t *idx, int count, c128 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((count + 255) / 256), dim3(256), 0, st, psi, idx, count, out);
  return hipGetLastError();
}

hipError_t launch_set_mat(c128 *dst, const c128 *m, int count, hipStream_t st) {
  Mat16 mm;
  for (int i = 0; i < 16; i++) mm.m[i] = i < count ? m[i] : make_double2(0, 0);
  hipLaunchKernelGGL(k_set_mat, dim3(1), dim3(16), 0, st, dst, mm, count);
  return hipGetLastError();
}

}  // namespace vqc

// Host side of the C ABI (include/vqc.h): validation, lowering of ops to
// register-level elementary ops, the fusion planner (HBM passes and register
// stages), device tables, and launch orchestration on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <deque>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vqc.h"
#include "jit.h"
#include "vqc_internal.h"

using namespace vqc;

namespace {

constexpr int kDefaultTile = 11;
constexpr int kDefaultAdjTile = 11;
constexpr int kDefaultLow = 4;
// plans of pure states with at least this many qubits move qubits into the
// low block between passes (fewer passes; a second state buffer for the
// forward, Phi and Psi each get one in the adjoint)
constexpr int kRemapMinBits = 12;
// the adjoint's moves need four states; above this many qubits its plan keeps
// the standard layout
constexpr int kAdjRemapMaxBits = 30;
// density matrices with at least this many vec(rho) bits run their forward and
// inverse-form adjoint on 11-bit LDS tiles (the 16x16 superoperator kind is
// compiled into that instantiation only)
constexpr int kMixedLdsMinBits = 12;
// pure-state plans with at least this many qubits get circuit-specialised
// forward passes compiled at run time (vqc_tune.jit = 0); below it a pass is
// too short for the compile to pay off and the interpreting kernel runs
constexpr int kJitMinBits = 20;
constexpr int kMixedTile = 11;
constexpr int kR = 4;

#define VQC_TRY(expr)                                         \
  do {                                                        \
    hipError_t _e = (expr);                                   \
    if (_e != hipSuccess) return hip_status(_e);              \
  } while (0)

vqc_status hip_status(hipError_t e) {
  if (e == hipSuccess) return VQC_OK;
  if (e == hipErrorOutOfMemory) return VQC_ERR_OOM;
  return VQC_ERR_HIP;
}

bool is_finite_d(double v) { return std::isfinite(v); }

// device allocation owned by a handle
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n && p) return hipSuccess;
    release();
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) { p = nullptr; return e; }
    n = bytes;
    return hipSuccess;
  }
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// ------------------------------------------------------------------ ops

int op_arity(int type) {
  if (type >= VQC_X && type <= VQC_ID) return 1;
  if (type >= VQC_CZ && type <= VQC_CONTROL) return 2;
  if (type >= VQC_TOFFOLI && type <= VQC_CCONTROL) return 3;
  if (type == VQC_AMPLITUDE_DAMPING || type == VQC_PHASE_DAMPING || type == VQC_DEPOLARIZING) return 1;
  if (type == VQC_DEPOLARIZING2) return 2;
  return 0;  // MATRIX, KRAUS: given by n_qubits
}
bool is_channel(int type) { return type >= VQC_AMPLITUDE_DAMPING && type <= VQC_KRAUS; }
int n_params_of(int type) {
  switch (type) {
    case VQC_RX: case VQC_RY: case VQC_RZ: case VQC_CRX: case VQC_CRY: case VQC_CRZ: return 1;
    case VQC_FSIM: return 5;
    default: return 0;
  }
}
bool valid_type(int t) {
  return (t >= VQC_X && t <= VQC_ID) || (t >= VQC_CZ && t <= VQC_CCONTROL) ||
         (t >= VQC_AMPLITUDE_DAMPING && t <= VQC_KRAUS);
}

// register kind of a gate matrix.  Structured kinds touch fewer FP64
// operations: real matrices (H, X, Ry), real-diagonal/imaginary-off-diagonal
// ones (Rx, Y), diagonal ones (Rz; Z, S, T change only the |1> half), fSim
// with Delta = 0.  sqrt(X), sqrt(Y), sqrt(W) are real/structured up to the
// global phase e^{i pi/4}; `factored` selects that form (pure states only).
int gate_kind(const vqc_op &op, bool factored) {
  const int type = op.type, m = op.n_qubits;
  if (m == 3) return GK_DENSE3;  // a general three-qubit matrix (named three-qubit gates are expanded)
  switch (type) {
    case VQC_Z: case VQC_S: case VQC_T: return GK_SPH1;
    case VQC_RZ: return GK_SDG1;
    case VQC_H: case VQC_X: return GK_REAL1;
    case VQC_RY: return GK_SRR1;
    case VQC_Y: return GK_XROT1;
    case VQC_RX: return GK_SXR1;
    case VQC_SX: return factored ? GK_SXR1 : GK_DENSE1;
    case VQC_SY: return factored ? GK_SRR1 : GK_DENSE1;
    case VQC_SW: return factored ? GK_SRD1 : GK_DENSE1;
    case VQC_ID: return GK_NONE;
    case VQC_CZ: case VQC_CRZ: return GK_DIAG2;
    case VQC_CNOT: return GK_CX;
    case VQC_FSIM: {
      bool plain = true;
      for (int k = 2; k < 5; k++) plain &= op.params[k] == 0.0 && op.param_index[k] < 0;
      return plain ? GK_SFX : GK_FSIM;
    }
    case VQC_SWAP: case VQC_ISWAP: return GK_FSIM;
    case VQC_CRX: case VQC_CRY: case VQC_CONTROL: return GK_DENSE2;
    case VQC_MATRIX: return m == 1 ? GK_DENSE1 : GK_DENSE2;
    default: return GK_DENSE1;
  }
}

// kinds applied from a shear record that follows the op's matrix
bool shear_kind(int gk) { return gk >= GK_SXR1 && gk <= GK_SFX; }

bool phase_factored(int type) { return type == VQC_SX || type == VQC_SY || type == VQC_SW; }

// row-major copy of a column-major ABI matrix
void to_row_major(const vqc_c128 *cm, int d, std::vector<c128> &out) {
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) out.push_back(make_double2(cm[r + d * c].re, cm[r + d * c].im));
}

vqc_status check_qubits(int m, const int *q, int n) {
  for (int i = 0; i < m; i++) {
    if (q[i] < 0 || q[i] >= n) return VQC_ERR_QUBIT;
    for (int j = 0; j < i; j++)
      if (q[i] == q[j]) return VQC_ERR_QUBIT;
  }
  return VQC_OK;
}

// sum_s K_s^dagger K_s == I within 1e-12 (column-major blocks)
bool kraus_complete(int m, int nk, const vqc_c128 *K) {
  const int d = 1 << m;
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) {
      double re = 0, im = 0;
      for (int s = 0; s < nk; s++) {
        const vqc_c128 *B = K + (size_t)s * d * d;
        for (int k = 0; k < d; k++) {
          // conj(K[k][r]) * K[k][c], element (row, col) at B[row + d col]
          const vqc_c128 a = B[k + d * r], b = B[k + d * c];
          re += a.re * b.re + a.im * b.im;
          im += a.re * b.im - a.im * b.re;
        }
      }
      if (std::fabs(re - (r == c ? 1.0 : 0.0)) > 1e-12 || std::fabs(im) > 1e-12) return false;
    }
  return true;
}

vqc_status validate_op(const vqc_op &op, int n, vqc_kind kind, int n_params) {
  if (!valid_type(op.type)) return VQC_ERR_ARG;
  const int ar = op_arity(op.type);
  const int m = op.n_qubits;
  if (m < 1 || m > 3) return VQC_ERR_UNSUPPORTED;
  // three qubits: the named gates, general matrices and Kraus sets (the last two as single ops only)
  if (m == 3 && op.type != VQC_MATRIX && op.type != VQC_KRAUS && ar != 3) return VQC_ERR_UNSUPPORTED;
  if (ar && ar != m) return VQC_ERR_ARG;
  vqc_status st = check_qubits(m, op.qubits, n);
  if (st) return st;
  if (is_channel(op.type) && kind != VQC_MIXED) return VQC_ERR_KIND;
  const int np = n_params_of(op.type);
  for (int k = 0; k < 5; k++) {
    if (!is_finite_d(op.params[k])) return VQC_ERR_NONFINITE;
    if (op.param_index[k] >= 0) {
      if (k >= np || op.param_index[k] >= n_params) return VQC_ERR_ARG;
    }
  }
  const int d = 1 << m;
  if (op.type == VQC_MATRIX) {
    if (!op.data || op.n_data != d * d) return VQC_ERR_ARG;
  } else if (op.type == VQC_CONTROL || op.type == VQC_CCONTROL) {
    if (!op.data || op.n_data != 4) return VQC_ERR_ARG;
  } else if (op.type == VQC_KRAUS) {
    if (!op.data || op.n_data <= 0 || op.n_data % (d * d) || op.n_data / (d * d) > 64) return VQC_ERR_ARG;
  }
  if (op.data)
    for (int i = 0; i < op.n_data; i++)
      if (!is_finite_d(op.data[i].re) || !is_finite_d(op.data[i].im)) return VQC_ERR_NONFINITE;
  if (op.type == VQC_KRAUS && !kraus_complete(m, op.n_data / (d * d), op.data)) return VQC_ERR_NOT_CPTP;
  if (op.type == VQC_AMPLITUDE_DAMPING || op.type == VQC_PHASE_DAMPING) {
    if (op.params[0] < 0 || op.params[0] > 1) return VQC_ERR_ARG;
  }
  if (op.type == VQC_DEPOLARIZING && (op.params[0] < 0 || op.params[0] > 4.0 / 3.0)) return VQC_ERR_ARG;
  if (op.type == VQC_DEPOLARIZING2 && (op.params[0] < 0 || op.params[0] > 16.0 / 15.0)) return VQC_ERR_ARG;
  return VQC_OK;
}

bool unitary_rm(const c128 *G, int d) {
  for (int r = 0; r < d; r++)
    for (int c = 0; c < d; c++) {
      double re = 0, im = 0;
      for (int k = 0; k < d; k++) {
        const c128 a = G[k * d + r], b = G[k * d + c];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
      }
      if (std::fabs(re - (r == c)) > 1e-10 || std::fabs(im) > 1e-10) return false;
    }
  return true;
}

// ------------------------------------------------------------ lowering

struct Deriv {
  int kind;
  int mat;
  int param;   // theta index
  int gslot;
};

struct Elem {
  int kind;
  int nq;
  int q[8];    // global bits (vec(rho) bits for mixed)
  int mat;     // matrix offset (c128 units), -1 if none
  bool inv = false;  // not unitary: its inverse is stored right after the matrix
  std::vector<Deriv> d;
  // GK_KRAUS3: offsets in the circuit's constant data of the Kraus set, its
  // adjoint set (K_s^dagger) and the inverse 64 x 64 superoperator; count
  int kd = -1, kda = -1, sinv = -1, nk = 0;
  // the unnormalised kind (GK_HX1..GK_HW1) the specialised forward passes
  // use for a phase-factored sqrt(X), sqrt(Y), sqrt(W), else 0
  int hk = 0;
  uint64_t mask() const {
    uint64_t m = 0;
    for (int i = 0; i < nq; i++) m |= 1ull << q[i];
    return m;
  }
};

struct PassH {
  int K;
  std::vector<int> tq;      // physical bit (input layout) of tile-local bit i, ascending
  std::vector<int> lq;      // logical qubit of tile-local bit i
  std::vector<int> tq_out;  // physical bit of tile-local bit i in the output layout
  bool moves = false;       // output layout differs from the input layout
  int src = 0, dst = 0;     // 0: the state's buffer, 1: the circuit's scratch state
  int lowfree = 0;          // DPass.lowfree as uploaded
  int special = -1;         // elem of a pass run by its own kernel (GK_KRAUS3), else -1
  int sk[3] = {0, 0, 0}, sb[3] = {0, 0, 0};  // its ket and bra bits in the pass's layout
  // a forward pass that moves qubits whose last stage's wave lanes cover the
  // new low set: the specialised kernel stores from registers
  bool jit_dout = false;
  struct Stage {
    int rbit[4];
    std::vector<int> elems;  // indices into elems
  };
  std::vector<Stage> stages;
};

struct Plan {
  bool reg_only = false;
  bool remap = false;          // passes move qubits between the low block and the rest
  bool d4 = false;             // LDS passes with 16x16 superoperators (density matrices)
  bool needs_scratch = false;  // some pass runs out of place
  int K = 0, R = kR, c = kDefaultLow;
  std::vector<PassH> passes;
  // device tables
  DevBuf dev;
  DPass *d_pass = nullptr;
  DJob *d_jobs1 = nullptr;  // single-item jobs, one per pass
  int n_stages = 0;
  int64_t units_per_item = 0;  // tiles (LDS) or blocks of 256 tiles (register-only)
  int prog = 0;                // c128 offset of the op program in an item's matrix buffer
  int n_gates = 0;
  const DGate *d_gates = nullptr;
  const DDeriv *d_derivs = nullptr;
  // circuit-specialised kernels of the passes (pure states): kernel p of this
  // plan is jit->fn[jit_base + p]; empty: the interpreting kernels run
  std::shared_ptr<JitModule> jit;
  int jit_base = 0;
  // LDS slots of every lane in every tile layout of the specialised forward
  // passes (see jit_source_fwd), read by those kernels
  DevBuf slots_buf;
  const uint16_t *d_slots = nullptr;
};

int popc(uint64_t v) { return __builtin_popcountll(v); }

// empty plan (keeps its device buffer for reuse)
void reset_plan(Plan &P) {
  P.passes.clear();
  P.reg_only = false;
  P.remap = false;
  P.d4 = false;
  P.needs_scratch = false;
  P.n_stages = 0;
  P.units_per_item = 0;
  P.prog = 0;
  P.n_gates = 0;
  P.d_pass = nullptr;
  P.d_jobs1 = nullptr;
  P.d_gates = nullptr;
  P.d_derivs = nullptr;
  P.jit.reset();
  P.d_slots = nullptr;
}

// First-fit fusion: walk the remaining ops in order; an op joins the pass if
// its qubits fit in the tile (<= K bits, the low c bits always included) and
// no earlier skipped op shares a qubit with it (program order on every qubit
// is kept, ops on disjoint qubits commute).  Then split each pass into
// register stages of R bits the same way.
// ops of `rem` (a prefix of at most `limit`) the first-fit rule takes into one
// tile of TK bits that must hold `forced`
int count_fit(const std::vector<Elem> &E, const std::vector<int> &rem, uint64_t forced, int TK, size_t limit) {
  uint64_t tile = forced, blocked = 0;
  int n = 0;
  for (size_t k = 0; k < rem.size() && k < limit; k++) {
    const uint64_t m = E[rem[k]].mask();
    if (m & blocked) { blocked |= m; continue; }
    if (popc(tile | m) <= TK) { tile |= m; n++; }
    else blocked |= m;
  }
  return n;
}

// Layout "low set first": the c qubits of L at physical bits 0..c-1 in
// ascending order, every other qubit after them in ascending order.
void layout_of(uint64_t L, int nbits, std::vector<int> &pos) {
  pos.assign(nbits, 0);
  int k = 0;
  for (int q = 0; q < nbits; q++)
    if ((L >> q) & 1) pos[q] = k++;
  for (int q = 0; q < nbits; q++)
    if (!((L >> q) & 1)) pos[q] = k++;
}

// the c-subset of `tile` that lets the next pass take the most ops
// (among the subsets that tie, one inside `prefer` if there is one)
uint64_t choose_low(const std::vector<Elem> &E, const std::vector<int> &rem, uint64_t tile, int c, int TK,
                    uint64_t prefer = 0) {
  std::vector<int> q;
  for (int b = 0; b < 64; b++)
    if ((tile >> b) & 1) q.push_back(b);
  const int t = (int)q.size();
  uint64_t best = 0;
  int best_n = -1;
  std::vector<int> idx(c);
  for (int i = 0; i < c; i++) idx[i] = i;
  while (true) {
    uint64_t L = 0;
    for (int i = 0; i < c; i++) L |= 1ull << q[idx[i]];
    const int n = count_fit(E, rem, L, TK, 256);
    if (n > best_n || (n == best_n && prefer && !(L & ~prefer) && (best & ~prefer))) {
      best_n = n;
      best = L;
    }
    int i = c - 1;
    while (i >= 0 && idx[i] == t - c + i) i--;
    if (i < 0) break;
    idx[i]++;
    for (int j = i + 1; j < c; j++) idx[j] = idx[j - 1] + 1;
  }
  return best;
}

// adjoint: the passes run in reverse, so a pass that moves qubits reads the
// layout the forward order leaves and writes the one it found; tile-local bits
// then follow the adjoint's input layout
void plan_passes(const std::vector<Elem> &E, int nbits, int K, int c, int R, bool reg_only, Plan &P,
                 int max_var, bool remap = false, bool adjoint = false) {
  P.passes.clear();
  P.reg_only = reg_only;
  P.remap = remap && !reg_only && c > 0;
  P.needs_scratch = false;
  P.K = reg_only ? R : K;
  P.R = R;
  P.c = c;
  std::vector<int> rem;
  for (size_t i = 0; i < E.size(); i++)
    if (E[i].kind != GK_NONE) rem.push_back((int)i);
  const int TK = reg_only ? R : K;
  // current layout: logical qubit -> physical bit; the low set L sits at bits 0..c-1
  const uint64_t home = reg_only ? 0 : ((1ull << c) - 1);
  uint64_t L = home;
  std::vector<int> pos, pos_next;
  layout_of(L, nbits, pos);
  auto finish_pass = [&](PassH &ph, uint64_t tile, const std::vector<int> &rest, uint64_t prefer) {
    uint64_t Ln = L;
    if (P.remap) {
      if (rest.empty()) Ln = ((home & ~tile) == 0) ? home : L;
      else Ln = choose_low(E, rest, tile, c, TK, prefer);
    }
    layout_of(Ln, nbits, pos_next);
    // tile-local bits in ascending position of the layout the kernel reads
    const std::vector<int> &pin = adjoint ? pos_next : pos, &pout = adjoint ? pos : pos_next;
    std::vector<int> qs;
    for (int b = 0; b < nbits; b++)
      if ((tile >> b) & 1) qs.push_back(b);
    std::sort(qs.begin(), qs.end(), [&](int x, int y) { return pin[x] < pin[y]; });
    ph.lq = qs;
    ph.tq.clear();
    ph.tq_out.clear();
    for (int q : qs) {
      ph.tq.push_back(pin[q]);
      ph.tq_out.push_back(pout[q]);
    }
    ph.moves = pos_next != pos;
    pos = pos_next;
    L = Ln;
  };
  while (!rem.empty()) {
    if (E[rem.front()].kind == GK_KRAUS3) {
      // a three-qubit channel: a pass of its own, in place, layout unchanged
      PassH ph;
      ph.K = 0;
      ph.special = rem.front();
      const Elem &e = E[ph.special];
      for (int t = 0; t < 3; t++) {
        ph.sk[t] = pos[e.q[t]];
        ph.sb[t] = pos[e.q[t + 3]];
      }
      P.passes.push_back(ph);
      rem.erase(rem.begin());
      continue;
    }
    uint64_t tile = reg_only ? 0 : L;
    uint64_t blocked = 0;
    int nvar = 0;
    std::vector<int> chosen, left;
    for (int i : rem) {
      const uint64_t m = E[i].mask();
      if (E[i].kind == GK_KRAUS3 || (m & blocked)) { blocked |= m; left.push_back(i); continue; }
      const uint64_t nt = tile | m;
      const int nd = (int)E[i].d.size();
      if (popc(nt) <= TK && (max_var <= 0 || nvar + nd <= max_var)) {
        tile = nt;
        nvar += nd;
        chosen.push_back(i);
      } else {
        blocked |= m;
        left.push_back(i);
      }
    }
    rem.swap(left);
    // pad the tile to exactly TK bits with the lowest unused bits
    for (int b = 0; b < nbits && popc(tile) < TK; b++) tile |= 1ull << b;
    PassH ph;
    ph.K = TK;
    // a forward pass's tile-local order follows the layout it reads, known
    // before the next layout is chosen: plan the stages first, so the next
    // low set can favour bits the last stage's wave lanes cover
    if (adjoint) {
      finish_pass(ph, tile, rem, 0);
    } else {
      ph.lq.clear();
      for (int b = 0; b < nbits; b++)
        if ((tile >> b) & 1) ph.lq.push_back(b);
      std::sort(ph.lq.begin(), ph.lq.end(), [&](int x, int y) { return pos[x] < pos[y]; });
    }
    int loc[64];
    for (int i = 0; i < (int)ph.lq.size(); i++) loc[ph.lq[i]] = i;
    // stages over tile-local bits: plain first fit, and a variant whose first
    // stage defers ops on the low c bits so it can read HBM directly; keep
    // the one with fewer LDS round trips
    const uint64_t lowloc = reg_only ? 0 : ((1ull << c) - 1);
    auto cost = [&](const std::vector<PassH::Stage> &st) {
      if (st.empty()) return 0;
      auto mask = [&](const PassH::Stage &S) {
        uint64_t m = 0;
        for (int i = 0; i < R; i++) m |= 1ull << S.rbit[i];
        return m;
      };
      return 2 * (int)st.size() + ((mask(st.front()) & lowloc) ? 1 : 0) + ((mask(st.back()) & lowloc) ? 1 : 0);
    };
    std::vector<PassH::Stage> best;
    std::vector<int> best_rest;
    // attempts 2 and 3 (unordered kinds only): each stage's register bits are
    // the R-subset of the tile's bits that takes the most of the remaining
    // ops (first fit restricted to the subset), the first stage of attempt 3
    // without low bits
    bool ordered_pass = false;
    for (int i : chosen) ordered_pass = ordered_pass || E[i].kind == GK_DENSE4 || E[i].kind == GK_DEPOL4;
    const int n_attempts = reg_only ? 1 : (ordered_pass ? 2 : 4);
    std::vector<uint64_t> subsets;
    if (n_attempts > 2) {
      for (uint64_t m = 0; m < (1ull << TK); m++)
        if (popc(m) == R) subsets.push_back(m);
    }
    auto local_mask = [&](int i) {
      uint64_t lm = 0;
      for (int t = 0; t < E[i].nq; t++) lm |= 1ull << loc[E[i].q[t]];
      return lm;
    };
    for (int attempt = 0; attempt < n_attempts; attempt++) {
      std::vector<PassH::Stage> stages;
      std::vector<int> srem = chosen, rest;
      bool failed = false;
      while (!srem.empty()) {
        uint64_t reg = 0, sblk = 0;
        if ((attempt == 1 || attempt == 3) && stages.empty()) sblk = lowloc;  // first stage: defer low bits
        uint64_t only = ~0ull;  // register bits a stage may use
        if (attempt >= 2) {
          int best_n = 0;
          for (uint64_t Q : subsets) {
            if (Q & sblk) continue;
            uint64_t blk = 0;
            int n = 0;
            for (int i : srem) {
              const uint64_t lm = local_mask(i);
              if (!(lm & blk) && !(lm & ~Q)) n++;
              else blk |= lm;
            }
            if (n > best_n) {
              best_n = n;
              only = Q;
            }
          }
          if (best_n == 0) only = ~0ull;
        }
        int order4[4] = {-1, -1, -1, -1};
        std::vector<int> st, sleft;
        for (int i : srem) {
          const uint64_t lm = local_mask(i);
          bool ok = !(lm & sblk) && !(lm & ~only) && popc(reg | lm) <= R;
          const bool ordered = E[i].kind == GK_DENSE4 || E[i].kind == GK_DEPOL4;  // register bits 0..3 in order
          if (ok && ordered) {
            if (order4[0] >= 0) {
              for (int t = 0; t < 4; t++)
                if (order4[t] != loc[E[i].q[t]]) ok = false;
            } else if (reg & ~lm) {
              ok = false;
            }
          }
          if (ok && order4[0] >= 0 && (lm & ~reg)) ok = false;
          if (!ok) { sblk |= lm; sleft.push_back(i); continue; }
          reg |= lm;
          st.push_back(i);
          if (ordered && order4[0] < 0)
            for (int t = 0; t < 4; t++) order4[t] = loc[E[i].q[t]];
        }
        if (st.empty()) {
          // nothing fitted (possible only when the first stage deferred the
          // low bits): this attempt is dropped
          if ((attempt == 1 || attempt == 3) && stages.empty()) { failed = true; break; }
          // an op wider than the register set cannot be planned; take it
          // alone so the loop always progresses (lowering never emits one)
          st.push_back(sleft.front());
          sleft.erase(sleft.begin());
          reg |= local_mask(st.back());
        }
        srem.swap(sleft);
        PassH::Stage S;
        if (order4[0] >= 0) {
          for (int t = 0; t < 4; t++) S.rbit[t] = order4[t];
        } else {
          if (only != ~0ull && popc(only) == R && !(reg & ~only)) reg = only;
          // pad with bits outside the low range first, so a stage stays low-free
          for (int b = TK - 1; b >= 0 && popc(reg) < R; b--)
            if (!((lowloc >> b) & 1) && !((reg >> b) & 1)) reg |= 1ull << b;
          for (int b = 0; b < TK && popc(reg) < R; b++) reg |= 1ull << b;
          int k = 0;
          for (int b = 0; b < TK; b++)
            if ((reg >> b) & 1) S.rbit[k++] = b;
        }
        S.elems = st;
        stages.push_back(S);
        if (reg_only && !srem.empty()) {
          rest = srem;
          break;
        }
      }
      if (failed) continue;
      if (best.empty() || cost(stages) < cost(best)) {
        best = stages;
        best_rest = rest;
      }
    }
    ph.stages = best;
    if (reg_only && !best_rest.empty()) {
      // register-only passes hold exactly one stage: push the rest back
      for (int i : best_rest) rem.push_back(i);
      std::sort(rem.begin(), rem.end());
    }
    if (!adjoint) {
      // the qubits at the last stage's six lowest lane bits (one wave's
      // lanes): a next low set among them lets the specialised kernel store
      // that stage's registers straight to HBM in the new layout, coalesced
      uint64_t prefer = 0;
      if (!ph.stages.empty() && !reg_only) {
        int nl = 0;
        for (int b = 0; b < TK && nl < 6; b++) {
          bool reg = false;
          for (int i = 0; i < R; i++) reg = reg || ph.stages.back().rbit[i] == b;
          if (reg) continue;
          prefer |= 1ull << ph.lq[b];
          nl++;
        }
      }
      finish_pass(ph, tile, rem, prefer);
      ph.jit_dout = ph.moves && prefer && !(L & ~prefer);
    }
    P.passes.push_back(ph);
  }
  if (!P.remap) return;
  auto empty_pass = [&]() {
    // a pass without ops whose tile holds the low set and the home low bits
    uint64_t tile = L | home;
    for (int b = 0; b < nbits && popc(tile) < TK; b++) tile |= 1ull << b;
    PassH ph;
    ph.K = TK;
    const std::vector<int> none;
    finish_pass(ph, tile, none, 0);
    P.passes.push_back(ph);
  };
  if (L != home) empty_pass();  // bring the layout back to the identity
  // A pass that changes the layout reads one buffer and writes the other;
  // the others may run in place.  The last pass must leave the state in
  // the caller's buffer, so the number of buffer switches must be even.
  int moving = 0;
  for (const PassH &ph : P.passes) moving += ph.moves;
  if (moving & 1) {
    bool fixed = false;
    for (PassH &ph : P.passes)
      if (!ph.moves && ph.special < 0) { ph.moves = true; fixed = true; break; }  // run one in-place pass out of place
    if (!fixed) {
      empty_pass();
      P.passes.back().moves = true;
    }
  }
  int cur = 0;
  for (PassH &ph : P.passes) {
    ph.src = cur;
    ph.dst = ph.moves ? 1 - cur : cur;
    cur = ph.dst;
    P.needs_scratch |= ph.moves;
  }
}

}  // namespace

// ------------------------------------------------------------- handles

struct vqc_state_s {
  vqc_kind kind;
  int n;
  int nbits;
  c128 *buf;
  hipStream_t stream;
  DevBuf mat;     // single-op matrices
  DevBuf red;     // expectation partials
  DevBuf small;   // jobs / terms / results
};

struct vqc_circuit_s {
  double jit_ms = 0;        // run-time compile (or cache load) of the specialised passes
  bool jit_cached = false;
  int live_batches = 0;     // batches holding pointers into this circuit's tables
  int n_special = 0;        // three-qubit channels (passes of their own)
  double special_kappa = 0; // their largest superoperator condition number
  int n, nbits;
  vqc_kind kind;
  int n_params;
  vqc_tune tune;
  std::vector<vqc_op> ops;
  std::vector<c128> cdata;
  std::vector<DRecipe> recipes;
  std::vector<DRecipe> subrec;  // one-qubit ops of fused runs (not built on their own)
  int mat_size = 0;   // recipe outputs
  int mat_total = 0;  // recipe outputs + op programs of both plans (c128 per item)
  std::vector<Elem> elems;
  int n_gslots = 0;
  std::vector<int> gslot_param;
  bool has_nonunitary_matrix = false;
  std::vector<DInv> inv_list;  // non-unitary ops (mixed): matrices to invert
  DevBuf dinv;                 // condition-number word, then inv_list
  Plan fwd, adj;   // pure: LDS forward + LDS adjoint; small mixed: register-only
  // mixed states of at least kMixedLdsMinBits vec(rho) bits: fwd and adj_lds
  // (inverse-form adjoint) on LDS tiles; adj and fwd_reg register-only with
  // one pass structure (the checkpointed adjoint and its forward recompute)
  Plan fwd_reg, adj_lds;
  DevBuf scratch;  // second state buffer for passes that move qubits (Phi in the adjoint)
  DevBuf scratch2; // second Psi buffer for adjoint passes that move qubits
  DevBuf dconst;   // recipes, constant data, csr
  DRecipe *d_rec = nullptr;
  c128 *d_cdata = nullptr;
  int32_t *d_csr_ptr = nullptr, *d_csr_slot = nullptr;
  DevBuf mats1;    // single-item matrices
  DevBuf psi1;     // single-item Psi (backward)
  DevBuf part1;    // single-item partials
  DevBuf ework;    // energy partials + result
  DevBuf ck;       // mixed checkpoints
  DevBuf small;
  int64_t adj_units = 0;
};

struct vqc_batch_s {
  int B;
  std::vector<vqc_circuit> circ;
  std::vector<c128 *> states;
  std::vector<const double *> thetas;
  hipStream_t stream;
  bool reg_only;
  int K, Kadj;
  int max_passes = 0, max_adj = 0;
  DevBuf mats, psi, part, tables, eparts, ck;
  std::vector<size_t> mat_off, psi_off, part_off;
  // second buffers of items whose passes move qubits: Phi (forward state), Psi
  DevBuf scr;
  std::vector<size_t> scr_off;
  // grouped build launches
  struct Group { vqc_circuit c; DevBuf ptrs; int count; };
  std::vector<std::unique_ptr<Group>> groups;
  DJob *d_fwd_jobs = nullptr;                 // concatenated per step
  std::vector<int> fwd_first, fwd_count;      // per step
  std::vector<int64_t> fwd_units;
  DJob *d_adj_jobs = nullptr;
  std::vector<int> adj_first, adj_count;
  std::vector<int64_t> adj_units;
  DEJob *d_ejobs = nullptr;                   // B expectation jobs (no out)
  DEJob *d_sjobs = nullptr;                   // B seed jobs (out = Psi)
  int64_t e_units = 0;
  DGradJob *d_gjobs = nullptr;
  int max_params = 0;
  double2 *d_eres = nullptr;
  DTerm *d_terms = nullptr;
  int n_terms = 0;
  std::vector<DTerm> terms_h;
  c128 **d_state_ptrs = nullptr;
  uint64_t *d_state_sizes = nullptr;
  bool built = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap_stream = nullptr;
  DevBuf kappa;  // largest condition number of the inverse-form backward
  // mixed batches: checkpoint layout
  int ck_stride = 0;
  std::vector<size_t> ck_off;  // per item: base offset into ck (bytes)
  size_t ck_per_item_states = 0;
};

namespace {

// ---------------------------------------------------------- circuit build

int add_recipe(vqc_circuit c, int type, int form, int k, int nq, const vqc_op &op, int data_off, int n_data,
               int out_size, int shear = 0) {
  DRecipe r;
  std::memset(&r, 0, sizeof(r));
  r.type = type;
  r.form = form;
  r.k = k;
  r.nq = nq;
  r.out = c->mat_size;
  r.data = data_off;
  r.n_data = n_data;
  r.shear = shear;
  for (int i = 0; i < 5; i++) {
    r.pidx[i] = op.param_index[i];
    r.pval[i] = op.params[i];
  }
  c->recipes.push_back(r);
  c->mat_size += out_size + (shear ? kSRecSlots : 0);
  return r.out;
}

// matrix of a gate op for the pass kernels: the offset the kernels read,
// i.e. the shear record for rotation kinds, the matrix otherwise
int add_gate_recipe(vqc_circuit c, int gk, int type, int form, int nq, const vqc_op &op, int data_off, int n_data) {
  const int d = 1 << nq;
  if (gk == GK_CX || gk == GK_NONE) return -1;
  if (shear_kind(gk)) return add_recipe(c, type, form, 0, nq, op, data_off, n_data, d * d, gk) + d * d;
  return add_recipe(c, type, form, 0, nq, op, data_off, n_data, d * d);
}

// room for the inverse of the D x D matrix just added at `mat`
void reserve_inverse(vqc_circuit c, int mat, int D) {
  DInv v;
  v.mat = mat;
  v.dim = D;
  c->inv_list.push_back(v);
  c->mat_size += D * D;
}

// a recipe for op `op` as a 4x4 superoperator of a fused run
DRecipe sub_recipe(const vqc_op &op, int data_off, int n_data) {
  DRecipe r;
  std::memset(&r, 0, sizeof(r));
  r.type = op.type;
  r.form = is_channel(op.type) ? RF_SUPER_KRAUS : RF_SUPER_GATE;
  r.nq = 1;
  r.data = data_off;
  r.n_data = n_data;
  for (int i = 0; i < 5; i++) {
    r.pidx[i] = op.param_index[i];
    r.pval[i] = op.params[i];
  }
  return r;
}

// A three-qubit Kraus set K_s (row-major 8 x 8 blocks at cdata[off]) as a
// special op: its adjoint set K_s^dagger (the adjoint superoperator is the
// Kraus sum of the K_s^dagger) and the inverse of its 64 x 64 superoperator
// S[(x + 8 y)][(x' + 8 y')] = sum_s K_s[x][x'] conj(K_s[y][y']) (Gauss-Jordan,
// partial pivoting), appended to the constant data; the 1-norm condition
// number ||S|| ||S^-1|| bounds the inverse-form sweep (infinite if singular).
void lower_kraus3(vqc_circuit c, const vqc_op &op, int off, int n_data, Elem &e) {
  using cd = std::complex<double>;
  const int nk = n_data / 64;
  std::vector<cd> K((size_t)nk * 64);
  for (int i = 0; i < nk * 64; i++) K[i] = cd(c->cdata[off + i].x, c->cdata[off + i].y);
  e.kind = GK_KRAUS3;
  e.nq = 6;
  const int n = c->n;
  for (int t = 0; t < 3; t++) {
    e.q[t] = op.qubits[t];
    e.q[t + 3] = op.qubits[t] + n;
  }
  e.mat = -1;
  e.kd = off;
  e.nk = nk;
  e.kda = (int)c->cdata.size();
  for (int k = 0; k < nk; k++)
    for (int r = 0; r < 8; r++)
      for (int col = 0; col < 8; col++) {
        const cd v = std::conj(K[k * 64 + col * 8 + r]);
        c->cdata.push_back(make_double2(v.real(), v.imag()));
      }
  std::vector<cd> S(4096, cd(0, 0)), A(4096), I(4096, cd(0, 0));
  for (int k = 0; k < nk; k++)
    for (int x = 0; x < 8; x++)
      for (int y = 0; y < 8; y++)
        for (int x2 = 0; x2 < 8; x2++)
          for (int y2 = 0; y2 < 8; y2++)
            S[(x + 8 * y) * 64 + (x2 + 8 * y2)] += K[k * 64 + x * 8 + x2] * std::conj(K[k * 64 + y * 8 + y2]);
  A = S;
  for (int i = 0; i < 64; i++) I[i * 64 + i] = 1.0;
  bool singular = false;
  for (int col = 0; col < 64 && !singular; col++) {
    int piv = col;
    for (int r = col + 1; r < 64; r++)
      if (std::abs(A[r * 64 + col]) > std::abs(A[piv * 64 + col])) piv = r;
    if (std::abs(A[piv * 64 + col]) == 0.0) { singular = true; break; }
    if (piv != col)
      for (int k = 0; k < 64; k++) {
        std::swap(A[piv * 64 + k], A[col * 64 + k]);
        std::swap(I[piv * 64 + k], I[col * 64 + k]);
      }
    const cd inv = 1.0 / A[col * 64 + col];
    for (int k = 0; k < 64; k++) {
      A[col * 64 + k] *= inv;
      I[col * 64 + k] *= inv;
    }
    for (int r = 0; r < 64; r++) {
      if (r == col) continue;
      const cd f = A[r * 64 + col];
      if (f == cd(0, 0)) continue;
      for (int k = 0; k < 64; k++) {
        A[r * 64 + k] -= f * A[col * 64 + k];
        I[r * 64 + k] -= f * I[col * 64 + k];
      }
    }
  }
  double kappa = std::numeric_limits<double>::infinity();
  if (!singular) {
    auto norm1 = [](const std::vector<cd> &M) {
      double best = 0;
      for (int col = 0; col < 64; col++) {
        double sum = 0;
        for (int r = 0; r < 64; r++) sum += std::abs(M[r * 64 + col]);
        best = std::max(best, sum);
      }
      return best;
    };
    kappa = norm1(S) * norm1(I);
    if (!std::isfinite(kappa)) kappa = std::numeric_limits<double>::infinity();
  }
  e.sinv = (int)c->cdata.size();
  for (int i = 0; i < 4096; i++) c->cdata.push_back(make_double2(singular ? 0.0 : I[i].real(), singular ? 0.0 : I[i].imag()));
  c->special_kappa = std::max(c->special_kappa, kappa);
  c->n_special++;
}

vqc_status lower(vqc_circuit c) {
  const int n = c->n;
  const bool mixed = c->kind == VQC_MIXED;
  int n_factored = 0;
  // constant data of every op (row-major)
  std::vector<int> doff(c->ops.size(), -1), ndat(c->ops.size(), 0);
  for (size_t j = 0; j < c->ops.size(); j++) {
    const vqc_op &op = c->ops[j];
    const int m = op.n_qubits, d = 1 << m;
    if (op.data && op.n_data > 0) {
      doff[j] = (int)c->cdata.size();
      if (op.type == VQC_CONTROL) {
        to_row_major(op.data, 2, c->cdata);  // the 2x2 target block
      } else {
        const int blocks = op.n_data / (d * d);
        for (int s = 0; s < blocks; s++) to_row_major(op.data + (size_t)s * d * d, d, c->cdata);
      }
      ndat[j] = op.n_data;
    }
    if (op.type == VQC_MATRIX && !unitary_rm(c->cdata.data() + doff[j], d)) c->has_nonunitary_matrix = true;
  }
  auto slot_for = [&](int param) {
    Deriv dv;
    dv.param = param;
    dv.gslot = c->n_gslots++;
    c->gslot_param.push_back(param);
    return dv;
  };
  for (size_t j = 0; j < c->ops.size(); j++) {
    const vqc_op &op = c->ops[j];
    const int m = op.n_qubits, d = 1 << m;
    const int data_off = doff[j], n_data = ndat[j];
    bool var = false;
    for (int k = 0; k < 5; k++) var |= op.param_index[k] >= 0;
    auto new_deriv = [&](int kind, int mat, int k) {
      Deriv dv = slot_for(op.param_index[k]);
      dv.kind = kind;
      dv.mat = mat;
      return dv;
    };
    if (mixed && m == 1) {
      // a run of one-qubit ops (gates and channels) on this qubit becomes one
      // 4x4 superoperator: S_{m-1} ... S_0, with one derivative per parameter
      size_t j2 = j + 1;
      while (j2 < c->ops.size() && c->ops[j2].n_qubits == 1 && c->ops[j2].qubits[0] == op.qubits[0]) j2++;
      if (j2 - j >= 2) {
        const int first = (int)c->subrec.size();
        for (size_t t = j; t < j2; t++) c->subrec.push_back(sub_recipe(c->ops[t], doff[t], ndat[t]));
        vqc_op none;
        std::memset(&none, 0, sizeof(none));
        for (int k = 0; k < 5; k++) none.param_index[k] = -1;
        Elem e;
        e.nq = 2;
        e.kind = GK_DENSE2;
        e.q[0] = op.qubits[0];
        e.q[1] = op.qubits[0] + n;
        e.mat = add_recipe(c, VQC_ID, RF_FUSED, 0, 1, none, first, (int)(j2 - j), 16);
        for (size_t t = j; t < j2; t++) e.inv = e.inv || is_channel(c->ops[t].type);
        if (e.inv) reserve_inverse(c, e.mat, 4);
        for (size_t t = j; t < j2; t++)
          for (int k = 0; k < 5; k++)
            if (c->ops[t].param_index[k] >= 0) {
              const int mat = add_recipe(c, VQC_ID, RF_DFUSED, (int)(t - j) * 8 + k, 1, none, first,
                                         (int)(j2 - j), 16);
              Deriv dv = slot_for(c->ops[t].param_index[k]);
              dv.kind = GK_DENSE2;
              dv.mat = mat;
              e.d.push_back(dv);
            }
        c->elems.push_back(e);
        j = j2 - 1;
        continue;
      }
    }
    if (is_channel(op.type) && m == 3) {
      Elem e;
      lower_kraus3(c, op, data_off, n_data, e);
      c->elems.push_back(e);
      continue;
    }
    if (is_channel(op.type)) {
      Elem e;
      e.nq = 2 * m;
      e.kind = m == 1 ? GK_DENSE2 : (op.type == VQC_DEPOLARIZING2 ? GK_DEPOL4 : GK_DENSE4);
      for (int t = 0; t < m; t++) { e.q[t] = op.qubits[t]; e.q[t + m] = op.qubits[t] + n; }
      e.mat = add_recipe(c, op.type, RF_SUPER_KRAUS, 0, m, op, data_off, n_data, d * d * d * d);
      e.inv = true;
      reserve_inverse(c, e.mat, d * d);
      c->elems.push_back(e);
      continue;
    }
    const int gk = gate_kind(op, !mixed);
    if (!mixed) {
      Elem e;
      e.nq = m;
      e.kind = gk;
      for (int t = 0; t < m; t++) e.q[t] = op.qubits[t];
      const bool fac = phase_factored(op.type);
      n_factored += fac;
      if (fac) e.hk = op.type == VQC_SX ? GK_HX1 : op.type == VQC_SY ? GK_HY1 : GK_HW1;
      e.mat = m == 3 ? add_recipe(c, op.type, RF_COPY, 0, m, op, data_off, n_data, d * d)
                     : add_gate_recipe(c, gk, op.type, fac ? RF_GATE_F : RF_GATE, m, op, data_off, n_data);
      // Pauli rotations exp(-i theta G / 2): derivative from the generator
      const int gen = op.type == VQC_RX ? GK_GENX : op.type == VQC_RY ? GK_GENY : op.type == VQC_RZ ? GK_GENZ : 0;
      for (int k = 0; k < 5; k++)
        if (op.param_index[k] >= 0) {
          if (gen) {
            e.d.push_back(new_deriv(gen, -1, k));
            continue;
          }
          const int dk = (m == 1) ? (gk == GK_SDG1 ? GK_DIAG1 : GK_DENSE1) : GK_DENSE2;
          const int mat = add_recipe(c, op.type, RF_DGATE, k, m, op, data_off, n_data, d * d);
          e.d.push_back(new_deriv(dk, mat, k));
        }
      c->elems.push_back(e);
    } else if (!var) {
      Elem e;
      e.nq = m;
      e.kind = gk;
      for (int t = 0; t < m; t++) e.q[t] = op.qubits[t];
      e.mat = m == 3 ? add_recipe(c, op.type, RF_COPY, 0, m, op, data_off, n_data, d * d)
                     : add_gate_recipe(c, gk, op.type, RF_GATE, m, op, data_off, n_data);
      c->elems.push_back(e);
      for (int t = 0; t < m; t++) e.q[t] = op.qubits[t] + n;
      e.mat = m == 3 ? add_recipe(c, op.type, RF_COPY, 1, m, op, data_off, n_data, d * d)
                     : add_gate_recipe(c, gk, op.type, RF_GATE_CONJ, m, op, data_off, n_data);
      c->elems.push_back(e);
    } else {
      Elem e;
      e.nq = 2 * m;
      e.kind = m == 1 ? GK_DENSE2 : GK_DENSE4;
      for (int t = 0; t < m; t++) { e.q[t] = op.qubits[t]; e.q[t + m] = op.qubits[t] + n; }
      e.mat = add_recipe(c, op.type, RF_SUPER_GATE, 0, m, op, data_off, n_data, d * d * d * d);
      for (int k = 0; k < 5; k++)
        if (op.param_index[k] >= 0) {
          const int mat = add_recipe(c, op.type, RF_DSUPER_GATE, k, m, op, data_off, n_data, d * d * d * d);
          e.d.push_back(new_deriv(e.kind, mat, k));
        }
      c->elems.push_back(e);
    }
  }
  if ((n_factored & 7) != 0) {
    // the product of the factored phases, e^{i pi n/4}, as one diagonal op
    vqc_op ph;
    std::memset(&ph, 0, sizeof(ph));
    for (int k = 0; k < 5; k++) ph.param_index[k] = -1;
    Elem e;
    e.nq = 1;
    e.kind = GK_SDG1;
    e.q[0] = 0;
    e.mat = add_recipe(c, VQC_ID, RF_GPHASE, n_factored & 7, 1, ph, -1, 0, 4, GK_SDG1) + 4;
    c->elems.push_back(e);
  }
  return VQC_OK;
}

// upload pass tables of a plan; single-item jobs reference no buffers (the
// kernel arguments supply them)
vqc_status upload_plan(vqc_circuit c, Plan &P, bool adjoint) {
  P.jit.reset();
  std::vector<DPass> passes(P.passes.size());
  std::vector<DStage> stages;
  std::vector<DGate> gates;
  std::vector<DDeriv> derivs;
  std::vector<int32_t> vslot;
  std::vector<int> pass_stage0, pass_deriv0, pass_vslot0;
  for (size_t p = 0; p < P.passes.size(); p++) {
    const PassH &ph = P.passes[p];
    int loc[64];
    for (int i = 0; i < (int)ph.lq.size(); i++) loc[ph.lq[i]] = i;
    pass_stage0.push_back((int)stages.size());
    pass_deriv0.push_back((int)derivs.size());
    pass_vslot0.push_back((int)vslot.size());
    int nvar = 0;
    for (const auto &S : ph.stages) {
      DStage ds;
      std::memset(&ds, 0, sizeof(ds));
      int srt[4];
      for (int i = 0; i < P.R; i++) { ds.rbit[i] = (int8_t)S.rbit[i]; srt[i] = S.rbit[i]; }
      std::sort(srt, srt + P.R);
      for (int i = 0; i < P.R; i++) ds.srt[i] = (int8_t)srt[i];
      ds.g0 = (int)gates.size();
      int regpos[64];
      for (int i = 0; i < P.R; i++) regpos[S.rbit[i]] = i;
      for (int ei : S.elems) {
        const Elem &e = c->elems[ei];
        DGate g;
        std::memset(&g, 0, sizeof(g));
        g.kind = (int8_t)e.kind;
        g.nq = (int8_t)e.nq;
        for (int t = 0; t < e.nq; t++) g.r[t] = (int8_t)regpos[loc[e.q[t]]];
        g.mat = e.mat;
        g.d0 = (int)derivs.size();
        g.nd = adjoint ? (int16_t)e.d.size() : 0;
        if (adjoint && !e.d.empty() && e.d[0].kind >= GK_GENX && e.d[0].kind <= GK_GENZ) g.nd |= kGenFlag;
        if (adjoint && e.inv) g.nd |= kInvFlag;
        if (adjoint)
          for (const Deriv &dv : e.d) {
            DDeriv dd;
            std::memset(&dd, 0, sizeof(dd));
            dd.kind = (int8_t)dv.kind;
            dd.mat = dv.mat;
            dd.gslot = dv.gslot;
            dd.local = nvar++;
            vslot.push_back(dv.gslot);
            derivs.push_back(dd);
          }
        gates.push_back(g);
      }
      ds.g1 = (int)gates.size();
      stages.push_back(ds);
    }
    if (nvar > kMaxVarPerPass) return VQC_ERR_UNSUPPORTED;
    DPass &dp = passes[p];
    std::memset(&dp, 0, sizeof(dp));
    dp.K = ph.K;
    dp.nst = (int)ph.stages.size();
    dp.nvar = nvar;
    dp.prog = P.prog;
    if (!P.reg_only && !ph.stages.empty()) {
      auto lowfree = [&](const PassH::Stage &S) {
        for (int i = 0; i < P.R; i++)
          if (S.rbit[i] < P.c) return false;
        return true;
      };
      // a pass that changes the layout stores through LDS (the output's low
      // bits are other tile bits than the input's); the adjoint stores after
      // the first stage in forward order
      const bool out_front = adjoint && ph.moves, out_back = !adjoint && ph.moves;
      dp.lowfree = ((lowfree(ph.stages.front()) && !out_front) ? 1 : 0) |
                   ((lowfree(ph.stages.back()) && !out_back) ? 2 : 0);
    }
    P.passes[p].lowfree = dp.lowfree;
    for (int i = 0; i < ph.K; i++) dp.tq[i] = (int8_t)ph.tq[i];
    // output order: tile-local bits by ascending output position
    std::vector<int> ord(ph.K);
    for (int i = 0; i < ph.K; i++) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return ph.tq_out[x] < ph.tq_out[y]; });
    for (int i = 0; i < ph.K; i++) {
      dp.lbo[i] = (int8_t)ord[i];
      dp.tqo[i] = (int8_t)ph.tq_out[ord[i]];
    }
  }
  P.n_stages = (int)stages.size();
  // one device blob: passes | jobs | stages | gates | derivs | vslot
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_pass = 0;
  const size_t o_jobs = al(o_pass + passes.size() * sizeof(DPass));
  const size_t o_st = al(o_jobs + passes.size() * sizeof(DJob));
  const size_t o_g = al(o_st + stages.size() * sizeof(DStage));
  const size_t o_d = al(o_g + gates.size() * sizeof(DGate));
  const size_t o_v = al(o_d + derivs.size() * sizeof(DDeriv));
  const size_t total = al(o_v + vslot.size() * sizeof(int32_t));
  VQC_TRY(P.dev.ensure(total));
  char *base = P.dev.as<char>();
  const int64_t tiles = int64_t(1) << (c->nbits - P.K);
  P.units_per_item = P.reg_only ? (tiles + 255) / 256 : tiles;
  std::vector<DJob> jobs(passes.size());
  for (size_t p = 0; p < passes.size(); p++) {
    passes[p].stages = reinterpret_cast<const DStage *>(base + o_st) + pass_stage0[p];
    passes[p].gates = reinterpret_cast<const DGate *>(base + o_g);
    passes[p].derivs = reinterpret_cast<const DDeriv *>(base + o_d);
    passes[p].vslot = reinterpret_cast<const int32_t *>(base + o_v) + pass_vslot0[p];
    DJob &j = jobs[p];
    std::memset(&j, 0, sizeof(j));
    j.pass = reinterpret_cast<const DPass *>(base + o_pass) + p;
    j.unit0 = 0;
    j.n_units = P.units_per_item;
    j.nbits = c->nbits;
  }
  std::vector<char> blob(total, 0);
  std::memcpy(blob.data() + o_pass, passes.data(), passes.size() * sizeof(DPass));
  std::memcpy(blob.data() + o_jobs, jobs.data(), jobs.size() * sizeof(DJob));
  std::memcpy(blob.data() + o_st, stages.data(), stages.size() * sizeof(DStage));
  std::memcpy(blob.data() + o_g, gates.data(), gates.size() * sizeof(DGate));
  std::memcpy(blob.data() + o_d, derivs.data(), derivs.size() * sizeof(DDeriv));
  std::memcpy(blob.data() + o_v, vslot.data(), vslot.size() * sizeof(int32_t));
  VQC_TRY(hipMemcpy(base, blob.data(), total, hipMemcpyHostToDevice));
  P.d_pass = reinterpret_cast<DPass *>(base + o_pass);
  P.d_jobs1 = reinterpret_cast<DJob *>(base + o_jobs);
  P.d_gates = reinterpret_cast<const DGate *>(base + o_g);
  P.d_derivs = reinterpret_cast<const DDeriv *>(base + o_d);
  P.n_gates = (int)gates.size();
  return VQC_OK;
}

// Source of the circuit-specialised forward passes of a pure-state LDS plan:
// for pass p a description JP<p> (tile and stage bit layouts, each op's kind
// and register bits, in program order) and the kernel vqc_jf<p>, which
// instantiates jit_pass.h's driver for it.  The op parameters stay in the
// item's op program, so one compiled plan serves every theta.
// LDS bank layout of a specialised pass's tile.  Local index l sits at slot
// (l & ~m) | N(l), m = 2^swb - 1 and N(l) the XOR of col[q] (swb bits) over
// the set bits q of l: a bijection, linear over XOR.  An access of
// consecutive lanes covers the banks once when the low bits of their slots
// differ, i.e. when the columns of their lowest varying bits are
// independent: for 16-byte elements (swb = 4) groups of 8 and of 16 lanes
// (32 or 64 banks), for 8-byte elements (swb = 5, a tile exchanged as real
// and imaginary halves) groups of 16 and 32.  The accesses are the stages'
// (lanes over the bits outside the stage's register bits), the tile's load
// (lanes over local bits 0..) and its store in the output layout (lanes over
// lbo[0..]).  col starts as the interpreter's fixed swizzle (low bits ^=
// bits 4..7 ^ bits 8..11) and a seeded random search replaces it when it
// finds fewer conflicting accesses.
std::vector<int> lds_swizzle(int K, int R, const PassH &ph, const std::vector<int> &lbo, int swb, uint64_t seed,
                             bool search = true) {
  std::vector<std::pair<std::vector<int>, int>> pats;  // lowest lane bits, accesses per lane
  auto lanes_of = [&](const std::vector<int> &bits, int w) {
    std::vector<int> v(bits.begin(), bits.begin() + std::min<size_t>(swb, bits.size()));
    pats.emplace_back(v, w);
  };
  std::vector<int> id;
  for (int q = 0; q < K - R; q++) id.push_back(q);
  lanes_of(id, 1 << R);
  lanes_of(std::vector<int>(lbo.begin(), lbo.begin() + (K - R)), 1 << R);
  for (const auto &S : ph.stages) {
    std::vector<int> lb;
    for (int q = 0; q < K; q++) {
      bool reg = false;
      for (int i = 0; i < R; i++) reg = reg || S.rbit[i] == q;
      if (!reg) lb.push_back(q);
    }
    lanes_of(lb, 2 << R);
  }
  auto indep = [](const int *v, int n, int mask) {
    int rows[8], nr = 0;
    for (int i = 0; i < n; i++) {
      int x = v[i] & mask;
      for (int r = 0; r < nr; r++) x = std::min(x, x ^ rows[r]);
      if (!x) return false;
      rows[nr++] = x;
      std::sort(rows, rows + nr, [](int a, int b) { return a > b; });
    }
    return true;
  };
  const int full = (1 << swb) - 1, part = (1 << (swb - 1)) - 1;
  auto cost = [&](const std::vector<int> &col) {
    int c = 0;
    for (const auto &pw : pats) {
      int v[8];
      const int n = (int)pw.first.size();
      for (int i = 0; i < n; i++) v[i] = col[pw.first[i]];
      if (!indep(v, n, full) || !indep(v, std::min(n, swb - 1), part)) c += pw.second;
    }
    return c;
  };
  std::vector<int> best(K);
  for (int q = 0; q < K; q++) best[q] = q < swb ? 1 << q : 1 << (q & 3);
  int bc = cost(best);
  uint64_t x = seed * 0x9e3779b97f4a7c15ull + 0x632be59bd9b4e019ull;
  std::vector<int> col(K);
  for (int it = 0; search && it < 6000 && bc > 0; it++) {
    for (int q = 0; q < K; q++) {
      x ^= x << 13;
      x ^= x >> 7;
      x ^= x << 17;
      col[q] = (int)(x >> 40) & full;
    }
    if (!indep(col.data(), std::min(K, swb), full)) continue;  // N must stay a bijection of each slot group
    const int cc = cost(col);
    if (cc < bc) {
      bc = cc;
      best = col;
    }
  }
  return best;
}

// the swizzle arrays of a pass description: SWC, SWB and SWDEF (SWC is the
// fixed fold l ^ ((l >> 4) ^ (l >> 8)) & 15, which the device computes in
// four instructions)
std::string swizzle_decl(const std::vector<int> &col, int swb) {
  bool def = swb == 4;
  for (size_t q = 0; q < col.size(); q++) def = def && col[q] == (q < 4 ? 1 << q : 1 << (q & 3)) && q < 12;
  std::string r = "  static constexpr int SWC[" + std::to_string(col.size()) + "] = {";
  for (size_t i = 0; i < col.size(); i++) r += (i ? ", " : "") + std::to_string(col[i]);
  r += "};\n  static constexpr int SWB = " + std::to_string(swb) + ";\n";
  r += def ? "  static constexpr bool SWDEF = true;\n" : "  static constexpr bool SWDEF = false;\n";
  return r;
}

// adjoint passes keep the fixed fold (measured faster: their per-lane slot
// arithmetic is not hoisted out of the stages); VQC_JIT_ADJ_SWZ=1 searches
// one per pass as the forward passes do
bool jit_adj_swizzle() {
  const char *e = std::getenv("VQC_JIT_ADJ_SWZ");
  return e && e[0] == '1';
}

// forward passes exchange the tile through LDS as real and imaginary halves
// (half the LDS per block, so more resident blocks, for two more barriers
// per stage change); VQC_JIT_FWD_SPLIT=0 keeps whole amplitudes
bool jit_fwd_split() {
  const char *e = std::getenv("VQC_JIT_FWD_SPLIT");
  return !(e && e[0] == '0');
}

// forward passes apply phase-factored sqrt(X), sqrt(Y), sqrt(W) unnormalised
// (GK_HX1..GK_HW1) and rescale the tile once; VQC_JIT_HSQRT=0 keeps the
// rotation forms
bool jit_fwd_hsqrt() {
  const char *e = std::getenv("VQC_JIT_HSQRT");
  return !(e && e[0] == '0');
}

// Lane slots of a forward pass: for each tile layout the kernel exchanges
// through LDS -- row 0 the load layout (lanes over the low tile bits), row
// 1 + S stage S's (lanes over the bits outside its register bits), row
// NST + 1 the store layout (lanes in output order) -- the byte offset in the
// LDS tile (elements of `width` bytes) of the swizzled slot of each lane's
// register 0, 2^(K-R) entries per row.  The kernel reads one entry per
// exchange instead of computing it.
void lane_slots(int K, int R, const PassH &ph, const std::vector<int> &lbo, const std::vector<int> &col, int swb,
                int width, std::vector<uint16_t> &tab) {
  const int T = 1 << (K - R), mask = (1 << swb) - 1;
  auto slot = [&](int l) {
    int n = 0;
    for (int q = 0; q < K; q++)
      if ((l >> q) & 1) n ^= col[q];
    return (uint16_t)(((l & ~mask) | n) * width);
  };
  for (int t = 0; t < T; t++) tab.push_back(slot(t));
  for (const auto &S : ph.stages) {
    int srt[4];
    for (int i = 0; i < R; i++) srt[i] = S.rbit[i];
    std::sort(srt, srt + R);
    for (int t = 0; t < T; t++) {
      int b = t;
      for (int i = 0; i < R; i++) b = ((b >> srt[i]) << (srt[i] + 1)) | (b & ((1 << srt[i]) - 1));
      tab.push_back(slot(b));
    }
  }
  for (int t = 0; t < T; t++) {
    int sl = 0;
    for (int i = 0; i < K - R; i++)
      if ((t >> i) & 1) sl |= 1 << lbo[i];
    tab.push_back(slot(sl));
  }
}

std::string jit_source_fwd(vqc_circuit c, const Plan &P, bool persist, std::string s, std::vector<uint16_t> &tab) {
  char buf[512];
  auto arr = [&](const char *name, const std::vector<int> &v) {
    std::string r = std::string("  static constexpr int ") + name + "[" + std::to_string(v.size()) + "] = {";
    for (size_t i = 0; i < v.size(); i++) r += (i ? ", " : "") + std::to_string(v[i]);
    return r + "};\n";
  };
  int g = 0;  // op index in the plan's program (upload_plan's order)
  for (size_t p = 0; p < P.passes.size(); p++) {
    const PassH &ph = P.passes[p];
    const int K = ph.K, R = P.R, nst = (int)ph.stages.size();
    int loc[64];
    for (int i = 0; i < (int)ph.lq.size(); i++) loc[ph.lq[i]] = i;
    std::vector<int> ord(K), tqo(K), lbo(K), tq(ph.tq.begin(), ph.tq.end());
    for (int i = 0; i < K; i++) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return ph.tq_out[x] < ph.tq_out[y]; });
    for (int i = 0; i < K; i++) {
      lbo[i] = ord[i];
      tqo[i] = ph.tq_out[ord[i]];
    }
    const bool split = jit_fwd_split();
    const bool hsq = jit_fwd_hsqrt();
    // program entries are read only by ops whose kind takes a record or a
    // matrix; each such op loads the entry of the next one (the pass's first
    // is loaded by the driver as G0)
    const char *rf = std::getenv("VQC_JIT_RECFREE");
    const bool recfree = !(rf && rf[0] == '0');
    std::vector<int> kinds, need;
    for (const auto &S : ph.stages)
      for (int ei : S.elems) {
        const Elem &e = c->elems[ei];
        kinds.push_back(hsq && e.hk ? e.hk : e.kind);
        const int k = kinds.back();
        need.push_back(!recfree || !(k == GK_CX || k == GK_HX1 || k == GK_HY1 || k == GK_HW1 || k == GK_NONE));
      }
    const int n_ops = (int)kinds.size();
    std::vector<int> next_need(n_ops + 1, g + std::max(n_ops - 1, 0));
    for (int k = n_ops - 1; k >= 0; k--) next_need[k] = need[k] ? g + k : next_need[k + 1];
    std::snprintf(buf, sizeof(buf),
                  "struct JP%zu {\n  static constexpr int K = %d, R = %d, NST = %d, PROG = %d, G0 = %d;\n"
                  "  static constexpr bool DIN = %s, DOUT = %s;\n",
                  p, K, R, nst, P.prog, next_need[0], (ph.lowfree & 1) ? "true" : "false",
                  ((ph.lowfree & 2) || ph.jit_dout) ? "true" : "false");
    s += buf;
    s += ph.moves ? "  static constexpr bool MOVES = true;\n" : "  static constexpr bool MOVES = false;\n";
    const int g_pass = g;
    int nh = 0;
    for (const auto &S : ph.stages)
      for (int ei : S.elems) nh += hsq && c->elems[ei].hk != 0;
    std::snprintf(buf, sizeof(buf), "  static constexpr int NH = %d;\n", nh);
    s += buf;
    const std::vector<int> col = lds_swizzle(K, R, ph, lbo, split ? 5 : 4, 2 * p + 1);
    std::snprintf(buf, sizeof(buf), "  static constexpr int TAB = %zu;\n", tab.size());
    s += buf;
    lane_slots(K, R, ph, lbo, col, split ? 5 : 4, split ? 8 : 16, tab);
    s += arr("TQ", tq) + arr("TQO", tqo) + arr("LBO", lbo) + arr("TQL", ph.tq_out) +
         swizzle_decl(col, split ? 5 : 4);
    const int rows = std::max(nst, 1);  // a pass without ops only moves qubits
    std::string rb = "  static constexpr int RBIT[" + std::to_string(rows) + "][" + std::to_string(R) + "] = {";
    std::string sr = "  static constexpr int SRT[" + std::to_string(rows) + "][" + std::to_string(R) + "] = {";
    if (nst == 0) {
      rb += "{0}";
      sr += "{0}";
    }
    for (int si = 0; si < nst; si++) {
      int srt[4];
      for (int i = 0; i < R; i++) srt[i] = ph.stages[si].rbit[i];
      std::sort(srt, srt + R);
      rb += si ? ", {" : "{";
      sr += si ? ", {" : "{";
      for (int i = 0; i < R; i++) {
        rb += (i ? ", " : "") + std::to_string(ph.stages[si].rbit[i]);
        sr += (i ? ", " : "") + std::to_string(srt[i]);
      }
      rb += "}";
      sr += "}";
    }
    s += rb + "};\n" + sr + "};\n";
    std::snprintf(buf, sizeof(buf),
                  "  template <int S>\n  __device__ static __forceinline__ DOp stage(c128 (&a)[%d], DOp E, "
                  "const DOp *prog, cmat *M) {\n",
                  1 << R);
    s += buf;
    for (int si = 0; si < nst; si++) {
      const PassH::Stage &S = ph.stages[si];
      int regpos[64];
      for (int i = 0; i < R; i++) regpos[S.rbit[i]] = i;
      s += si ? "    else if constexpr (S == " : "    if constexpr (S == ";
      s += std::to_string(si) + ") {\n";
      for (int ei : S.elems) {
        const Elem &e = c->elems[ei];
        const int b0 = e.nq > 0 ? regpos[loc[e.q[0]]] : 0, b1 = e.nq > 1 ? regpos[loc[e.q[1]]] : 0;
        const int b2 = e.nq > 2 ? regpos[loc[e.q[2]]] : 0;
        const int k = g - g_pass, kind = kinds[k];
        if (need[k])
          std::snprintf(buf, sizeof(buf), "      E = jop<%d, %d, %d, %d, %d>(a, E, prog + %d, M);\n", R, kind, b0,
                        b1, b2, next_need[k + 1]);
        else
          std::snprintf(buf, sizeof(buf), "      jopn<%d, %d, %d, %d>(a);\n", R, kind, b0, b1);
        s += buf;
        g++;
      }
      s += "      return E;\n    }\n";
    }
    s += nst ? "    else return E;\n  }\n};\n" : "    return E;\n  }\n};\n";
    std::snprintf(buf, sizeof(buf),
                  "extern \"C\" __global__ void __launch_bounds__(%d) vqc_jf%zu(const DJob *__restrict__ jobs, "
                  "int n_jobs, int64_t total_units, DOverride ov, const uint16_t *__restrict__ slots) {\n"
                  "  jit_pass_fwd<JP%zu, %s, %s>(jobs, n_jobs, total_units, ov, slots);\n}\n",
                  1 << (K - R), p, p, persist ? "true" : "false", split ? "true" : "false");
    s += buf;
  }
  return s;
}

// Source of the specialised adjoint passes of a pure-state LDS plan (Alg. 2):
// description JA<p> with its stages' ops in reverse program order, each op
// with its derivative reductions (generator form before Phi is uncomputed,
// derivative matrices after), and the kernel vqc_ja<p>.
// adjoint driver (VQC_JIT_ADJ_SPLIT): 1 (default) jit_pass_adj2, lane slots
// from the table and the tile exchanged as real and imaginary halves; 2 the
// same with whole amplitudes; 0 jit_pass_adj (lane slots computed, fixed
// fold, VQC_JIT_ADJ_SHARED / VQC_JIT_ADJ_SWZ apply)
int jit_adj_driver() {
  const char *e = std::getenv("VQC_JIT_ADJ_SPLIT");
  return e && (e[0] == '0' || e[0] == '2') ? e[0] - '0' : 1;
}

std::string jit_source_adj(vqc_circuit c, const Plan &P, bool shared, std::string s, std::vector<uint16_t> &tab) {
  const int drv = jit_adj_driver();
  char buf[512];
  auto arr = [&](const char *name, const std::vector<int> &v) {
    std::string r = std::string("  static constexpr int ") + name + "[" + std::to_string(std::max<size_t>(1, v.size())) +
                    "] = {";
    for (size_t i = 0; i < v.size(); i++) r += (i ? ", " : "") + std::to_string(v[i]);
    if (v.empty()) r += "0";
    return r + "};\n";
  };
  int g = 0;  // program index of the next op (upload_plan's order)
  for (size_t p = 0; p < P.passes.size(); p++) {
    const PassH &ph = P.passes[p];
    const int K = ph.K, R = P.R, nst = (int)ph.stages.size(), T = 1 << (K - R);
    const int WS = T < 64 ? T : 64, NW = (T + 63) / 64;
    int loc[64];
    for (int i = 0; i < (int)ph.lq.size(); i++) loc[ph.lq[i]] = i;
    std::vector<int> ord(K), tqo(K), lbo(K), tq(ph.tq.begin(), ph.tq.end());
    for (int i = 0; i < K; i++) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return ph.tq_out[x] < ph.tq_out[y]; });
    for (int i = 0; i < K; i++) {
      lbo[i] = ord[i];
      tqo[i] = ph.tq_out[ord[i]];
    }
    // derivative slots in forward order, as the uploaded tables number them
    std::vector<int> vslot;
    std::vector<std::vector<int>> slots;  // per op of the pass, in program order
    int n_ops = 0;
    for (const auto &S : ph.stages)
      for (int ei : S.elems) {
        slots.emplace_back();
        for (const Deriv &dv : c->elems[ei].d) {
          slots.back().push_back((int)vslot.size());
          vslot.push_back(dv.gslot);
        }
        n_ops++;
      }
    const int g0 = g;
    // execution order (stages and their ops in reverse); ops of kinds that
    // read no program entry (controlled X) skip the entry chain, each other op
    // loading the entry of the next such op
    std::vector<int> first_op(nst + 1, 0);
    for (int si = 0; si < nst; si++) first_op[si + 1] = first_op[si] + (int)ph.stages[si].elems.size();
    std::vector<int> exec_gi, exec_need;
    for (int si = nst - 1; si >= 0; si--)
      for (int q = (int)ph.stages[si].elems.size() - 1; q >= 0; q--) {
        const int kind = c->elems[ph.stages[si].elems[q]].kind;
        exec_gi.push_back(g0 + first_op[si] + q);
        exec_need.push_back(!(kind == GK_CX || kind == GK_NONE));
      }
    std::vector<int> next_exec(exec_gi.size() + 1, g0 + std::max(n_ops - 1, 0));
    for (int k = (int)exec_gi.size() - 1; k >= 0; k--) next_exec[k] = exec_need[k] ? exec_gi[k] : next_exec[k + 1];
    std::vector<int> exec_pos(n_ops, 0);
    for (size_t k = 0; k < exec_gi.size(); k++) exec_pos[exec_gi[k] - g0] = (int)k;
    std::snprintf(buf, sizeof(buf),
                  "struct JA%zu {\n  static constexpr int K = %d, R = %d, NST = %d, PROG = %d, GLAST = %d, NVAR = %d;\n"
                  "  static constexpr int WS = %d, NW = %d;\n"
                  "  static constexpr bool DIN = %s, DOUT = %s;\n",
                  p, K, R, nst, P.prog, next_exec[0], (int)vslot.size(), WS, NW,
                  (ph.lowfree & 2) ? "true" : "false", (ph.lowfree & 1) ? "true" : "false");
    s += buf;
    if (drv == 0) {
      s += arr("TQ", tq) + arr("TQO", tqo) + arr("LBO", lbo) + arr("VSLOT", vslot) +
           swizzle_decl(lds_swizzle(K, R, ph, lbo, 4, 2 * p + 2, jit_adj_swizzle()), 4);
    } else {
      const int swb = drv == 1 ? 5 : 4;
      const std::vector<int> col = lds_swizzle(K, R, ph, lbo, swb, 2 * p + 2);
      std::snprintf(buf, sizeof(buf), "  static constexpr int TAB = %zu;\n", tab.size());
      s += buf;
      lane_slots(K, R, ph, lbo, col, swb, drv == 1 ? 8 : 16, tab);
      s += arr("TQ", tq) + arr("TQO", tqo) + arr("LBO", lbo) + arr("VSLOT", vslot) + swizzle_decl(col, swb);
    }
    const int rows = std::max(nst, 1);
    std::string rb = "  static constexpr int RBIT[" + std::to_string(rows) + "][" + std::to_string(R) + "] = {";
    std::string sr = "  static constexpr int SRT[" + std::to_string(rows) + "][" + std::to_string(R) + "] = {";
    if (nst == 0) {
      rb += "{0}";
      sr += "{0}";
    }
    for (int si = 0; si < nst; si++) {
      int srt[4];
      for (int i = 0; i < R; i++) srt[i] = ph.stages[si].rbit[i];
      std::sort(srt, srt + R);
      rb += si ? ", {" : "{";
      sr += si ? ", {" : "{";
      for (int i = 0; i < R; i++) {
        rb += (i ? ", " : "") + std::to_string(ph.stages[si].rbit[i]);
        sr += (i ? ", " : "") + std::to_string(srt[i]);
      }
      rb += "}";
      sr += "}";
    }
    s += rb + "};\n" + sr + "};\n";
    std::snprintf(buf, sizeof(buf),
                  "  template <int S>\n  __device__ static __forceinline__ DOp astage(c128 (&a)[%d], c128 (&b)[%d], "
                  "DOp E, const DOp *prog, cmat *M, double (*red)[%d], int lane, int wave) {\n",
                  1 << R, 1 << R, NW);
    s += buf;
    int k = 0;  // op of the pass in program order
    std::vector<int> first_k(nst + 1, 0);
    for (int si = 0; si < nst; si++) first_k[si + 1] = first_k[si] + (int)ph.stages[si].elems.size();
    for (int si = 0; si < nst; si++) {
      const PassH::Stage &S = ph.stages[si];
      int regpos[64];
      for (int i = 0; i < R; i++) regpos[S.rbit[i]] = i;
      s += si ? "    else if constexpr (S == " : "    if constexpr (S == ";
      s += std::to_string(si) + ") {\n";
      for (int q = (int)S.elems.size() - 1; q >= 0; q--) {
        const Elem &e = c->elems[S.elems[q]];
        k = first_k[si] + q;
        const int gi = g0 + k;
        const int b0 = e.nq > 0 ? regpos[loc[e.q[0]]] : 0, b1 = e.nq > 1 ? regpos[loc[e.q[1]]] : 0;
        const int b2 = e.nq > 2 ? regpos[loc[e.q[2]]] : 0;
        const bool gen = !e.d.empty() && e.d[0].kind >= GK_GENX && e.d[0].kind <= GK_GENZ;
        const int xp = exec_pos[gi - g0];
        if (!exec_need[xp]) {
          std::snprintf(buf, sizeof(buf),
                        "      {\n        __builtin_amdgcn_sched_barrier(0);\n"
                        "        japply<R, true, %d, %d, %d, %d>(a, E, M);\n        japply<R, true, %d, %d, %d, %d>(b, E, M);\n"
                        "        __builtin_amdgcn_sched_barrier(0);\n      }\n",
                        e.kind, b0, b1, b2, e.kind, b0, b1, b2);
          s += buf;
          continue;
        }
        std::snprintf(buf, sizeof(buf),
                      "      {\n        lgkm_wait();\n        const DOp En = ldc(prog + %d);\n"
                      "        __builtin_amdgcn_sched_barrier(0);\n",
                      next_exec[xp + 1]);
        s += buf;
        if (gen) {
          std::snprintf(buf, sizeof(buf),
                        "        jred<WS, NW>(red, %d, jgrad<R, %d, %d, 0>(a, b, M), lane, wave);\n", slots[k][0],
                        (int)e.d[0].kind, b0);
          s += buf;
        }
        std::snprintf(buf, sizeof(buf), "        japply<R, true, %d, %d, %d, %d>(a, E, M);\n", e.kind, b0, b1, b2);
        s += buf;
        if (!gen)
          for (size_t d = 0; d < e.d.size(); d++) {
            std::snprintf(buf, sizeof(buf),
                          "        jred<WS, NW>(red, %d, jgrad<R, %d, %d, %d>(a, b, M + %d), lane, wave);\n",
                          slots[k][d], (int)e.d[d].kind, b0, b1, e.d[d].mat);
            s += buf;
          }
        std::snprintf(buf, sizeof(buf),
                      "        japply<R, true, %d, %d, %d, %d>(b, E, M);\n        E = En;\n"
                      "        __builtin_amdgcn_sched_barrier(0);\n      }\n",
                      e.kind, b0, b1, b2);
        s += buf;
      }
      s += "      return E;\n    }\n";
    }
    s += nst ? "    else return E;\n  }\n};\n" : "    return E;\n  }\n};\n";
    g = g0 + n_ops;
    std::snprintf(buf, sizeof(buf),
                  "extern \"C\" __global__ void __launch_bounds__(%d) vqc_ja%zu(const DJob *__restrict__ jobs, "
                  "int n_jobs, int64_t total_units, DOverride ov, const uint16_t *slots) {\n  %s",
                  T, p, "");
    s += buf;
    if (drv == 0)
      std::snprintf(buf, sizeof(buf), "jit_pass_adj<JA%zu, %s>(jobs, n_jobs, total_units, ov);\n}\n", p,
                    shared ? "true" : "false");
    else
      std::snprintf(buf, sizeof(buf), "jit_pass_adj2<JA%zu, %s>(jobs, n_jobs, total_units, ov, slots);\n}\n", p,
                    drv == 1 ? "true" : "false");
    s += buf;
  }
  return s;
}

// whether a pure-state circuit asks for circuit-specialised forward passes
// (vqc_tune.jit; VQC_JIT=0 / 1 in the environment turns them off / on for
// every eligible plan)
bool jit_default_on(vqc_circuit c) {
  if (c->kind != VQC_PURE) return false;
  if (const char *e = std::getenv("VQC_JIT")) {
    if (e[0] == '0') return false;
    if (e[0] == '1') return true;
  }
  if (c->tune.jit < 0) return false;
  return c->tune.jit > 0 || c->nbits >= kJitMinBits;
}

bool jit_wanted(vqc_circuit c) {
  const Plan &P = c->fwd;
  if (c->kind != VQC_PURE || P.reg_only || P.d4 || P.passes.empty() || P.K > 11) return false;
  return jit_default_on(c);
}

bool jit_plan_ok(const Plan &P) { return !P.reg_only && !P.d4 && !P.passes.empty() && P.K <= 11; }

// compile (or load from the cache) the specialised forward and adjoint passes
// of a pure-state circuit, one module for both plans; a failure leaves the
// interpreting kernels in charge unless the caller asked for these kernels
// (vqc_tune.jit = 1)
vqc_status jit_prepare(vqc_circuit c, bool with_adj = true) {
  c->fwd.jit.reset();
  c->adj.jit.reset();
  c->fwd.d_slots = nullptr;
  c->adj.d_slots = nullptr;
  c->jit_ms = 0;
  if (!jit_wanted(c)) return VQC_OK;
  // persistent grids when the caller asked for a grid size (vqc_tune.grid_blocks)
  const bool persist = c->tune.grid_blocks > 0;
  const bool adj = with_adj && jit_plan_ok(c->adj) && c->adj.K <= 10 + (c->adj.R == 3 ? 1 : 0);
  std::vector<std::string> names;
  std::vector<int> threads;
  std::string src = "#include \"jit_pass.h\"\nnamespace vqc {\n";
  std::vector<uint16_t> tab;
  src = jit_source_fwd(c, c->fwd, persist, src, tab);
  for (size_t p = 0; p < c->fwd.passes.size(); p++) {
    names.push_back("vqc_jf" + std::to_string(p));
    threads.push_back(1 << (c->fwd.passes[p].K - c->fwd.R));
  }
  if (adj) {
    // Phi and Psi share one LDS tile (set VQC_JIT_ADJ_SHARED=0 for one each)
    const char *sh = std::getenv("VQC_JIT_ADJ_SHARED");
    src = jit_source_adj(c, c->adj, !(sh && sh[0] == '0'), src, tab);
    for (size_t p = 0; p < c->adj.passes.size(); p++) {
      names.push_back("vqc_ja" + std::to_string(p));
      threads.push_back(1 << (c->adj.passes[p].K - c->adj.R));
    }
  }
  src += "}  // namespace vqc\n";
  if (const char *dump = std::getenv("VQC_JIT_DUMP")) {  // keep the generated source for inspection
    if (FILE *f = std::fopen((std::string(dump) + "/vqc_jit_" + std::to_string(c->n) + ".hip").c_str(), "w")) {
      std::fputs(src.c_str(), f);
      std::fclose(f);
    }
  }
  std::shared_ptr<JitModule> m(new (std::nothrow) JitModule());
  if (!m) return VQC_ERR_OOM;
  std::string log;
  const hipError_t e = jit_build(src, names, threads, *m, &log);
  if (e != hipSuccess) {
    if (std::getenv("VQC_JIT_VERBOSE")) std::fprintf(stderr, "vqc: run-time compile failed:\n%s\n", log.c_str());
    return c->tune.jit > 0 ? VQC_ERR_HIP : VQC_OK;
  }
  const size_t nf = c->fwd.passes.size();
  for (size_t k = 0; k < m->resident.size(); k++) {
    if (k < nf && persist) m->resident[k] = std::min(m->resident[k], c->tune.grid_blocks);
    else m->resident[k] = 0x7fffffff;  // one block per tile
  }
  {
    hipError_t ue = c->fwd.slots_buf.ensure(tab.size() * sizeof(uint16_t));
    if (ue == hipSuccess)
      ue = hipMemcpy(c->fwd.slots_buf.p, tab.data(), tab.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
    if (ue != hipSuccess) return c->tune.jit > 0 ? VQC_ERR_HIP : VQC_OK;
  }
  c->jit_ms = m->ms;
  c->jit_cached = m->cached;
  c->fwd.jit = m;
  c->fwd.jit_base = 0;
  c->fwd.d_slots = c->fwd.slots_buf.as<uint16_t>();
  if (adj) {
    c->adj.jit = m;
    c->adj.jit_base = (int)nf;
    c->adj.d_slots = c->fwd.d_slots;  // the adjoint's rows follow the forward's in one table
  }
  return VQC_OK;
}

vqc_status make_plans(vqc_circuit c) {
  const bool mixed = c->kind == VQC_MIXED;
  const int nb = c->nbits;
  int K = c->tune.tile_bits > 0 ? c->tune.tile_bits : kDefaultTile;
  int low = c->tune.low_bits > 0 ? c->tune.low_bits : kDefaultLow;
  if (K > kMaxTile) K = kMaxTile;
  const bool mixed_lds = mixed && nb >= kMixedLdsMinBits;
  const bool reg_only = (mixed && !mixed_lds) || nb < 5;
  int R = std::min(kR, nb);
  // the adjoint step keeps two states and runs derivative reductions: three
  // register bits (more waves per SIMD) beat four there, while four are best
  // for the forward pass (measured on the 20-qubit gradient and the
  // 28-qubit circuit)
  int Radj = (!reg_only && nb >= 8) ? 3 : R;
  if (!reg_only && c->tune.reg_bits == 3) {
    R = 3;
    Radj = 3;
  }
  // specialised forward passes run best with three register bits (more waves
  // per SIMD; measured on the 28-qubit circuit: 45.6 ms against 48.8 ms with
  // four), the interpreting kernel with four
  if (!reg_only && !mixed && c->tune.reg_bits == 0 && jit_default_on(c)) R = 3;
  // op programs follow the recipe outputs in each item's matrix buffer
  reset_plan(c->fwd_reg);
  reset_plan(c->adj_lds);
  c->fwd.d4 = c->adj.d4 = false;
  c->fwd.prog = c->mat_size;
  auto prog_end = [](const Plan &P) { return P.prog + (P.n_gates + 2) * kOpSlots; };
  if (mixed_lds) {
    const int lowm = std::min(low, kMixedTile - 4);  // a two-qubit superoperator spans 4 bits
    const bool remap = c->tune.remap > 0 || (c->tune.remap == 0 && nb >= kRemapMinBits);
    plan_passes(c->elems, nb, kMixedTile, lowm, 4, false, c->fwd, 0, remap);
    c->fwd.d4 = true;
    vqc_status st = upload_plan(c, c->fwd, false);
    if (st) return st;
    c->adj.prog = prog_end(c->fwd);
    plan_passes(c->elems, nb, 4, 0, 4, true, c->adj, kMaxVarPerPass);
    st = upload_plan(c, c->adj, true);
    if (st) return st;
    c->fwd_reg.prog = prog_end(c->adj);
    plan_passes(c->elems, nb, 4, 0, 4, true, c->fwd_reg, kMaxVarPerPass);
    st = upload_plan(c, c->fwd_reg, false);
    if (st) return st;
    c->adj_lds.prog = prog_end(c->fwd_reg);
    plan_passes(c->elems, nb, kMixedTile, lowm, 4, false, c->adj_lds, kMaxVarPerPass,
                remap && nb <= kAdjRemapMaxBits, true);
    c->adj_lds.d4 = true;
    st = upload_plan(c, c->adj_lds, true);
    if (st) return st;
  } else if (reg_only) {
    plan_passes(c->elems, nb, R, 0, R, true, c->fwd, kMaxVarPerPass);
    vqc_status st = upload_plan(c, c->fwd, false);
    if (st) return st;
    c->adj.prog = c->fwd.prog + (c->fwd.n_gates + 2) * kOpSlots;
    plan_passes(c->elems, nb, R, 0, R, true, c->adj, kMaxVarPerPass);
    st = upload_plan(c, c->adj, true);
    if (st) return st;
  } else {
    const int kmin = R == 3 ? 8 : 5;
    if (nb < kmin) { R = Radj = 4; }
    K = std::max(R == 3 ? 8 : 5, std::min(K, nb));
    // the low block plus any two-qubit op must fit in a tile
    low = std::min(low, K - 2);
    int Ka = std::max(Radj == 3 ? 8 : 5, std::min(std::min(K, kDefaultAdjTile), nb));
    const bool remap = c->tune.remap > 0 || (c->tune.remap == 0 && nb >= kRemapMinBits);
    plan_passes(c->elems, nb, K, low, R, false, c->fwd, 0, remap);
    vqc_status st = upload_plan(c, c->fwd, false);
    if (st) return st;
    c->adj.prog = c->fwd.prog + (c->fwd.n_gates + 2) * kOpSlots;
    plan_passes(c->elems, nb, Ka, std::min(low, Ka - 2), Radj, false, c->adj, kMaxVarPerPass,
                remap && nb <= kAdjRemapMaxBits, true);
    st = upload_plan(c, c->adj, true);
    if (st) return st;
  }
  c->mat_total = std::max(prog_end(c->adj), c->adj_lds.passes.empty() ? 0 : prog_end(c->adj_lds));
  if (c->mats1.ensure((size_t)c->mat_total * sizeof(c128)) != hipSuccess) return VQC_ERR_HIP;
  if ((c->fwd.needs_scratch || c->adj.needs_scratch || c->adj_lds.needs_scratch) &&
      c->scratch.ensure((size_t(1) << nb) * sizeof(c128)) != hipSuccess)
    return VQC_ERR_OOM;
  c->tune.tile_bits = c->fwd.K;
  c->tune.low_bits = c->fwd.c;
  c->tune.reg_bits = c->fwd.R;
  if (c->tune.remap == 0) c->tune.remap = c->fwd.remap ? 1 : -1;
  return VQC_OK;
}

vqc_status upload_const(vqc_circuit c) {
  // recipes | cdata | csr_ptr | csr_slot
  std::vector<int32_t> ptr(c->n_params + 1, 0), slot;
  std::vector<std::vector<int>> per(c->n_params);
  for (int s = 0; s < c->n_gslots; s++) per[c->gslot_param[s]].push_back(s);
  for (int p = 0; p < c->n_params; p++) {
    ptr[p + 1] = ptr[p] + (int)per[p].size();
    for (int s : per[p]) slot.push_back(s);
  }
  // fused runs refer to their sub-recipes, stored after the built recipes
  std::vector<DRecipe> rec = c->recipes;
  for (DRecipe &r : rec)
    if (r.form == RF_FUSED || r.form == RF_DFUSED) r.data += (int)c->recipes.size();
  rec.insert(rec.end(), c->subrec.begin(), c->subrec.end());
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t o_r = 0, o_c = al(rec.size() * sizeof(DRecipe));
  const size_t o_p = al(o_c + c->cdata.size() * sizeof(c128));
  const size_t o_s = al(o_p + ptr.size() * sizeof(int32_t));
  const size_t total = al(o_s + slot.size() * sizeof(int32_t));
  VQC_TRY(c->dconst.ensure(total));
  std::vector<char> blob(total, 0);
  std::memcpy(blob.data() + o_r, rec.data(), rec.size() * sizeof(DRecipe));
  std::memcpy(blob.data() + o_c, c->cdata.data(), c->cdata.size() * sizeof(c128));
  std::memcpy(blob.data() + o_p, ptr.data(), ptr.size() * sizeof(int32_t));
  std::memcpy(blob.data() + o_s, slot.data(), slot.size() * sizeof(int32_t));
  char *base = c->dconst.as<char>();
  VQC_TRY(hipMemcpy(base, blob.data(), total, hipMemcpyHostToDevice));
  c->d_rec = reinterpret_cast<DRecipe *>(base + o_r);
  c->d_cdata = reinterpret_cast<c128 *>(base + o_c);
  c->d_csr_ptr = reinterpret_cast<int32_t *>(base + o_p);
  c->d_csr_slot = reinterpret_cast<int32_t *>(base + o_s);
  VQC_TRY(c->mats1.ensure((size_t)c->mat_total * sizeof(c128)));
  if (!c->inv_list.empty()) {
    VQC_TRY(c->dinv.ensure(256 + c->inv_list.size() * sizeof(DInv)));
    VQC_TRY(hipMemcpy(c->dinv.as<char>() + 256, c->inv_list.data(), c->inv_list.size() * sizeof(DInv),
                      hipMemcpyHostToDevice));
  }
  return VQC_OK;
}

// terms with i^{|Y|} folded into the coefficient
// term t of H with i^{|Y|} folded into its coefficient
vqc_status make_term(const vqc_pauli_sum *H, int t, int nbits_q, bool need_real, DTerm &d) {
  const uint64_t xm = H->x_mask[t], zm = H->z_mask[t];
  if (nbits_q < 64 && ((xm | zm) >> nbits_q)) return VQC_ERR_QUBIT;
  double cr = H->coeff_re[t], ci = H->coeff_im ? H->coeff_im[t] : 0.0;
  if (!is_finite_d(cr) || !is_finite_d(ci)) return VQC_ERR_NONFINITE;
  if (need_real && ci != 0.0) return VQC_ERR_NOT_HERMITIAN;
  const int ny = popc(xm & zm) & 3;
  double r = cr, i = ci;
  for (int k = 0; k < ny; k++) { const double tr = -i; i = r; r = tr; }  // multiply by i
  d.xm = xm;
  d.zm = zm;
  d.cre = r;
  d.cim = i;
  return VQC_OK;
}

bool pauli_sum_ok(const vqc_pauli_sum *H) {
  return H && H->n_terms >= 0 && (H->n_terms == 0 || (H->x_mask && H->z_mask && H->coeff_re));
}

vqc_status make_terms(const vqc_pauli_sum *H, int nbits_q, std::vector<DTerm> &out, bool need_real) {
  if (!pauli_sum_ok(H)) return VQC_ERR_ARG;
  out.clear();
  for (int t = 0; t < H->n_terms; t++) {
    DTerm d;
    const vqc_status st = make_term(H, t, nbits_q, need_real, d);
    if (st) return st;
    out.push_back(d);
  }
  return VQC_OK;
}

int grid_of(vqc_circuit c, int64_t units) {
  const int g = c->tune.grid_blocks;
  if (g > 0 && g < units) return g;
  return (int)std::min<int64_t>(units, int64_t(1) << 30);
}

// forward plan whose passes line up with the register-only adjoint (the
// checkpointed mixed backward recomputes states pass by pass)
Plan &ck_fwd(vqc_circuit c) { return c->fwd_reg.passes.empty() ? c->fwd : c->fwd_reg; }
// adjoint plan of the inverse-form mixed backward (and of batches)
Plan &inv_adj(vqc_circuit c) { return c->adj_lds.passes.empty() ? c->adj : c->adj_lds; }
Plan &batch_adj(vqc_circuit c) { return c->kind == VQC_MIXED ? inv_adj(c) : c->adj; }

// matrices, rotation records and the op programs of every plan for B items
// (thetas / mats per item) or one item (theta0 / mats0)
hipError_t build_mats(vqc_circuit c, const double *const *thetas, c128 *const *mats, int B, const double *theta0,
                      c128 *mats0, hipStream_t st) {
  hipError_t e = launch_build_mats(c->d_rec, (int)c->recipes.size(), c->d_cdata, thetas, mats, B, theta0, mats0, st);
  if (e != hipSuccess) return e;
  e = launch_assemble(c->fwd.d_gates, c->fwd.d_derivs, c->fwd.n_gates, c->fwd.prog, mats, B, mats0, st);
  if (e != hipSuccess) return e;
  for (const Plan *P : {&c->fwd_reg, &c->adj_lds})
    if (!P->passes.empty()) {
      e = launch_assemble(P->d_gates, P->d_derivs, P->n_gates, P->prog, mats, B, mats0, st);
      if (e != hipSuccess) return e;
    }
  return launch_assemble(c->adj.d_gates, c->adj.d_derivs, c->adj.n_gates, c->adj.prog, mats, B, mats0, st);
}

// one specialised pass: a block per tile of every job (the driver is not
// persistent), static LDS
hipError_t launch_jit_pass(const JitModule &m, size_t p, const Plan &P, const DJob *jobs, int n_jobs, int64_t total,
                           const DOverride &ov, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  const size_t k = P.jit_base + p;
  if (p >= P.passes.size() || k >= m.fn.size() || k >= m.resident.size()) return hipErrorInvalidValue;
  const int64_t grid = std::min<int64_t>(total, m.resident[k]);
  DOverride o = ov;
  const uint16_t *slots = P.d_slots;
  void *args[] = {&jobs, &n_jobs, &total, &o, &slots};
  return hipModuleLaunchKernel(m.fn[k], (unsigned)grid, 1, 1, 1u << (P.passes[p].K - P.R), 1, 1, 0, st, args,
                               nullptr);
}

// run passes [p0, p1) of a plan on one item (dir > 0: forward order)
// mode 0: forward in place (b == nullptr) or a -> b; 1: pure adjoint; 2: mixed adjoint
hipError_t run_passes(vqc_circuit c, Plan &P, int mode, c128 *a, c128 *b, const c128 *mats, double *partials,
                      int p0, int p1, int dir, hipStream_t st) {
  DOverride ov;
  ov.a = a;
  ov.b = b;
  ov.a2 = nullptr;
  ov.b2 = nullptr;
  ov.mats = mats;
  ov.partials = partials;
  ov.mode = (mode == 0 && b) ? 1 : 0;
  ov.use = 1;
  ov.job_units = 0;
  const int grid = grid_of(c, P.units_per_item);
  // passes that move qubits alternate between the state and the circuit's
  // scratch state (the plan ends in the state); the adjoint runs the plan
  // backwards with Phi and Psi, so it reads a pass's destination and writes
  // its source
  const bool pingpong = P.needs_scratch && ((mode == 0 && !b) || mode == 1);
  c128 *bufs[2] = {a, c->scratch.as<c128>()};
  c128 *bufb[2] = {b, c->scratch2.as<c128>()};
  for (int k = 0; k < p1 - p0; k++) {
    const int p = dir > 0 ? p0 + k : p1 - 1 - k;
    if (P.passes[p].special >= 0) {
      // a three-qubit channel (its own kernel, in place; the layout is the
      // same before and after, so the current buffers are the pass's source)
      const PassH &ph = P.passes[p];
      const Elem &e = c->elems[ph.special];
      const c128 *cd = c->d_cdata;
      c128 *phi = pingpong ? (mode == 0 ? bufs[ph.src] : bufs[ph.dst]) : a;
      c128 *psi = pingpong && mode != 0 ? bufb[ph.dst] : b;
      hipError_t e2 = hipSuccess;
      if (mode == 0) {
        if (b && !pingpong) {  // out of place: the channel on a copy
          e2 = launch_copy(b, a, uint64_t(1) << c->nbits, st);
          phi = b;
        }
        if (e2 == hipSuccess) e2 = launch_block6(phi, c->nbits, ph.sk, ph.sb, cd + e.kd, e.nk, 0, st);
      } else {
        // Phi <- M^{-1} Phi (inverse forms), Psi <- M^dagger Psi (every form;
        // the adjoint of the Kraus sum is the sum over the K_s^dagger)
        if (mode == 1 || mode == 3) e2 = launch_block6(phi, c->nbits, ph.sk, ph.sb, cd + e.sinv, 0, 1, st);
        if (e2 == hipSuccess) e2 = launch_block6(psi, c->nbits, ph.sk, ph.sb, cd + e.kda, e.nk, 0, st);
      }
      if (e2 != hipSuccess) return e2;
      continue;
    }
    if (pingpong) {
      const PassH &ph = P.passes[p];
      if (mode == 0) {
        ov.a = bufs[ph.src];
        ov.b = bufs[ph.dst];
      } else {
        ov.a = bufs[ph.dst];
        ov.b = bufb[ph.dst];
        ov.a2 = bufs[ph.src];
        ov.b2 = bufb[ph.src];
      }
      ov.mode = ph.src != ph.dst ? 1 : 0;
    }
    hipError_t e;
    if ((mode == 0 || mode == 1) && P.jit) e = launch_jit_pass(*P.jit, p, P, P.d_jobs1 + p, 1, P.units_per_item, ov, st);
    else if (P.reg_only) e = launch_pass_reg(P.R, mode, P.d_jobs1 + p, 1, P.units_per_item, grid, ov, st);
    else e = launch_pass_lds(P.K, P.R, mode != 0, P.d4, P.d_jobs1 + p, 1, P.units_per_item, grid, ov, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

uint64_t state_len(vqc_kind kind, int n) { return kind == VQC_MIXED ? (1ull << (2 * n)) : (1ull << n); }

}  // namespace

// ===================================================================== C ABI

// ------------------------------------------- scratch of the allocation-free
// expectation (vqc_expectation_noalloc).  One fixed array per GPU, held for
// the life of the process: first-stage partial sums, the Pauli terms, the
// job record and the result.  In host code `scratch` names a host-side
// stand-in; kernels get the device address returned by hipGetSymbolAddress.
constexpr int64_t kNaMaxUnits = int64_t(1) << 16;  // partials: 2^16 x 4096 = 2^28 amplitudes
constexpr int kNaMaxTerms = 1024;
constexpr size_t kNaTermOff = size_t(kNaMaxUnits) * sizeof(double2);
constexpr size_t kNaJobOff = kNaTermOff + size_t(kNaMaxTerms) * sizeof(DTerm);
constexpr size_t kNaResOff = kNaJobOff + 256;
constexpr size_t kNaBytes = kNaResOff + 256;
static_assert(sizeof(DEJob) <= 256, "job record must fit its slot");
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
char *g_na_ptr[kNaMaxDevices] = {};

// device address of `scratch` on the GPU that runs `st`, looked up once per
// device with that device current
hipError_t na_scratch(hipStream_t st, char **out) {
  int dev = 0;
  hipError_t e = hipStreamGetDevice(st, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = (cur != dev) ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    if (!p) return hipErrorInvalidSymbol;
    g_na_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_na_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

const char *vqc_status_string(int st) {
  switch (st) {
    case VQC_OK: return "ok";
    case VQC_ERR_ARG: return "invalid argument";
    case VQC_ERR_QUBIT: return "qubit out of range or repeated";
    case VQC_ERR_UNSUPPORTED: return "unsupported op or combination";
    case VQC_ERR_KIND: return "pure/mixed state kind mismatch";
    case VQC_ERR_NOT_CPTP: return "Kraus operators are not trace preserving";
    case VQC_ERR_NONFINITE: return "non-finite input";
    case VQC_ERR_OOM: return "device out of memory";
    case VQC_ERR_HIP: return "HIP runtime error";
    case VQC_ERR_NOT_HERMITIAN: return "observable must have real coefficients";
    case VQC_ERR_NOT_UNITARY: return "gate matrix is not unitary";
    case VQC_ERR_ILL_CONDITIONED: return "channel inverse exceeds the condition-number bound";
    case VQC_ERR_SCRATCH_LIMIT: return "input exceeds the fixed scratch of the allocation-free call";
    case VQC_ERR_IN_USE: return "circuit is bound to a live batch";
    default: return "unknown status";
  }
}

int vqc_version(void) { return 100; }

vqc_status vqc_mat_from_external(int m, const vqc_c128 *rm, vqc_c128 *out) {
  if (m < 1 || m > 4 || !rm || !out) return VQC_ERR_ARG;
  const int d = 1 << m;
  auto rev = [m](int x) {
    int r = 0;
    for (int t = 0; t < m; t++)
      if ((x >> t) & 1) r |= 1 << (m - 1 - t);
    return r;
  };
  for (int lo = 0; lo < d; lo++)
    for (int li = 0; li < d; li++) out[lo + d * li] = rm[rev(lo) * d + rev(li)];
  return VQC_OK;
}

// --------------------------------------------------------------- states

vqc_status vqc_state_init(vqc_state *out, vqc_kind kind, int n, void *dev_buf, const vqc_c128 *host_init,
                          void *stream) {
  if (!out || !dev_buf) return VQC_ERR_ARG;
  if (kind != VQC_PURE && kind != VQC_MIXED) return VQC_ERR_ARG;
  if (n < 1 || (kind == VQC_PURE && n > 33) || (kind == VQC_MIXED && n > 16)) return VQC_ERR_ARG;
  const uint64_t N = state_len(kind, n);
  if (host_init)
    for (uint64_t i = 0; i < N; i++)
      if (!is_finite_d(host_init[i].re) || !is_finite_d(host_init[i].im)) return VQC_ERR_NONFINITE;
  vqc_state s = new (std::nothrow) vqc_state_s();
  if (!s) return VQC_ERR_OOM;
  s->kind = kind;
  s->n = n;
  s->nbits = kind == VQC_MIXED ? 2 * n : n;
  s->buf = reinterpret_cast<c128 *>(dev_buf);
  s->stream = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = s->mat.ensure(512 * sizeof(c128));
  if (e == hipSuccess) {
    if (host_init) {
      e = hipMemcpyAsync(s->buf, host_init, N * sizeof(c128), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    } else {
      e = launch_init_basis0(s->buf, N, s->stream);
    }
  }
  if (e != hipSuccess) {
    delete s;
    return hip_status(e);
  }
  *out = s;
  return VQC_OK;
}

vqc_status vqc_state_reset(vqc_state s) {
  if (!s) return VQC_ERR_ARG;
  VQC_TRY(launch_init_basis0(s->buf, state_len(s->kind, s->n), s->stream));
  return VQC_OK;
}

vqc_status vqc_state_rebind(vqc_state s, void *dev_buf, void *stream) {
  if (!s || !dev_buf) return VQC_ERR_ARG;
  s->buf = reinterpret_cast<c128 *>(dev_buf);
  s->stream = reinterpret_cast<hipStream_t>(stream);
  return VQC_OK;
}

vqc_status vqc_state_destroy(vqc_state s) {
  delete s;
  return VQC_OK;
}

static bool is_zero(const c128 &v) { return v.x == 0.0 && v.y == 0.0; }
static bool is_one(const c128 &v) { return v.x == 1.0 && v.y == 0.0; }

// structure of a row-major gate matrix for the single-op kernels
static int single_kind(int m, const c128 *G) {
  if (m == 1) {
    if (is_zero(G[1]) && is_zero(G[2])) return is_one(G[0]) ? SK_PHASE1 : SK_DIAG1;
    return SK_DENSE1;
  }
  bool diag = true, ctrl = true, fsim = true;
  for (int r = 0; r < 4; r++)
    for (int c = 0; c < 4; c++) {
      const bool z = is_zero(G[r * 4 + c]);
      if (r != c && !z) diag = false;
      const bool in_ctrl = (r & 1) && (c & 1);
      if (!in_ctrl && !((r == c) ? is_one(G[r * 4 + c]) : z)) ctrl = false;
      const bool in_f = (r == c) || (r == 1 && c == 2) || (r == 2 && c == 1);
      if (!in_f && !z) fsim = false;
    }
  if (diag) return (is_one(G[0]) && is_one(G[5]) && is_one(G[10])) ? SK_PHASE11 : SK_DIAG2;
  if (ctrl) {
    if (is_zero(G[5]) && is_one(G[7]) && is_one(G[13]) && is_zero(G[15])) return SK_CX;
    return SK_CTRL;
  }
  if (fsim && is_one(G[0])) return SK_FSIM;
  return SK_DENSE2;
}

static hipError_t apply_single(vqc_state s, int m, const int *q, const c128 *dev_mat, int kind) {
  if (m == 1) return launch_g1(s->buf, s->nbits, q[0], dev_mat, kind, s->stream);
  if (m == 3) return launch_gm(s->buf, s->nbits, 3, q, dev_mat, s->stream);
  return launch_g2(s->buf, s->nbits, q[0], q[1], dev_mat, kind, s->stream);
}

// the 8x8 matrix (ABI column-major) of a three-qubit gate type
static void gate3_matrix(const vqc_op &o, vqc_c128 *cm) {
  std::memset(cm, 0, 64 * sizeof(vqc_c128));
  for (int l = 0; l < 8; l++) {  // column l (input), local index b0 + 2 b1 + 4 b2
    if (o.type == VQC_TOFFOLI) {
      cm[((l & 3) == 3 ? l ^ 4 : l) + 8 * l].re = 1;
    } else if (o.type == VQC_FREDKIN) {
      const bool sw = (l & 1) && (((l >> 1) & 1) != ((l >> 2) & 1));
      cm[(sw ? l ^ 6 : l) + 8 * l].re = 1;
    } else {  // CCONTROL: column-major 2x2 data u[out + 2 in] on bit 2
      if ((l & 3) != 3) {
        cm[l + 8 * l].re = 1;
        continue;
      }
      const int b = l >> 2;
      cm[3 + 8 * l] = o.data[0 + 2 * b];
      cm[7 + 8 * l] = o.data[1 + 2 * b];
    }
  }
}

vqc_status vqc_apply_gate(vqc_state s, int m, const int *qubits, const vqc_c128 *matrix) {
  if (!s || !qubits || !matrix) return VQC_ERR_ARG;
  if (m < 1 || m > 3) return VQC_ERR_UNSUPPORTED;
  vqc_status st = check_qubits(m, qubits, s->n);
  if (st) return st;
  const int d = 1 << m;
  for (int i = 0; i < d * d; i++)
    if (!is_finite_d(matrix[i].re) || !is_finite_d(matrix[i].im)) return VQC_ERR_NONFINITE;
  std::vector<c128> G;
  to_row_major(matrix, d, G);
  if (m == 3) {
    // dense 8x8 (Alg. 1 with three nested strides): U, then conj(U) on the bra bits
    c128 *dm = s->mat.as<c128>();
    std::vector<c128> both(G);
    for (const c128 &v : G) both.push_back(make_double2(v.x, -v.y));
    VQC_TRY(hipMemcpyAsync(dm, both.data(), both.size() * sizeof(c128), hipMemcpyHostToDevice, s->stream));
    VQC_TRY(apply_single(s, 3, qubits, dm, 0));
    if (s->kind == VQC_MIXED) {
      const int qb[3] = {qubits[0] + s->n, qubits[1] + s->n, qubits[2] + s->n};
      VQC_TRY(apply_single(s, 3, qb, dm + 64, 0));
    }
    VQC_TRY(hipStreamSynchronize(s->stream));  // the host source is local
    return VQC_OK;
  }
  const int kind = single_kind(m, G.data());
  c128 *dm = s->mat.as<c128>();
  VQC_TRY(launch_set_mat(dm, G.data(), d * d, s->stream));
  VQC_TRY(apply_single(s, m, qubits, dm, kind));
  if (s->kind == VQC_MIXED) {
    // rho -> U rho U^dagger: conj(U) on the bra bits
    std::vector<c128> Gc(G);
    for (auto &v : Gc) v.y = -v.y;
    int qb[2] = {qubits[0] + s->n, m > 1 ? qubits[1] + s->n : 0};
    VQC_TRY(launch_set_mat(dm + 16, Gc.data(), d * d, s->stream));
    VQC_TRY(apply_single(s, m, qb, dm + 16, kind));
  }
  return VQC_OK;
}

static int typed_kind(int type) {
  switch (type) {
    case VQC_Z: case VQC_S: case VQC_T: return SK_PHASE1;
    case VQC_RZ: return SK_DIAG1;
    case VQC_CZ: return SK_PHASE11;
    case VQC_CNOT: return SK_CX;
    case VQC_SWAP: case VQC_ISWAP: case VQC_FSIM: return SK_FSIM;
    case VQC_CRX: case VQC_CRY: case VQC_CRZ: return SK_CTRL;
    default: return op_arity(type) == 2 ? SK_DENSE2 : SK_DENSE1;
  }
}

static vqc_status apply_channel_dev(vqc_state s, int m, const int *q, int type, double prm, const std::vector<c128> &kraus_rm,
                                    int n_data);

vqc_status vqc_apply_op(vqc_state s, const vqc_op *op) {
  if (!s || !op) return VQC_ERR_ARG;
  vqc_op o = *op;
  for (int k = 0; k < 5; k++) o.param_index[k] = -1;  // values, not variational slots
  vqc_status st = validate_op(o, s->n, s->kind, 0);
  if (st) return st;
  const int m = o.n_qubits, d = 1 << m;
  if (is_channel(o.type)) {
    std::vector<c128> K;
    if (o.type == VQC_KRAUS)
      for (int b = 0; b < o.n_data / (d * d); b++) to_row_major(o.data + (size_t)b * d * d, d, K);
    return apply_channel_dev(s, m, o.qubits, o.type, o.params[0], K, o.n_data);
  }
  if (o.type == VQC_MATRIX) return vqc_apply_gate(s, m, o.qubits, o.data);
  if (m == 3) {
    vqc_c128 full[64];
    gate3_matrix(o, full);
    return vqc_apply_gate(s, 3, o.qubits, full);
  }
  if (o.type == VQC_CONTROL) {
    vqc_c128 full[16];
    std::memset(full, 0, sizeof(full));
    full[0 + 4 * 0].re = 1;
    full[2 + 4 * 2].re = 1;
    // column-major (out, in) at [out + 4 in]; control=1 block at local 1, 3
    full[1 + 4 * 1] = o.data[0 + 2 * 0];
    full[1 + 4 * 3] = o.data[0 + 2 * 1];
    full[3 + 4 * 1] = o.data[1 + 2 * 0];
    full[3 + 4 * 3] = o.data[1 + 2 * 1];
    return vqc_apply_gate(s, 2, o.qubits, full);
  }
  if (o.type == VQC_ID) return VQC_OK;
  DRecipe r;
  std::memset(&r, 0, sizeof(r));
  r.type = o.type;
  r.form = RF_GATE;
  r.nq = m;
  r.data = -1;
  for (int k = 0; k < 5; k++) { r.pidx[k] = -1; r.pval[k] = o.params[k]; }
  c128 *dm = s->mat.as<c128>();
  const int kind = typed_kind(o.type);
  VQC_TRY(launch_build_one(r, nullptr, dm, s->stream));
  VQC_TRY(apply_single(s, m, o.qubits, dm, kind));
  if (s->kind == VQC_MIXED) {
    r.form = RF_GATE_CONJ;
    VQC_TRY(launch_build_one(r, nullptr, dm + 16, s->stream));
    int qb[2] = {o.qubits[0] + s->n, m > 1 ? o.qubits[1] + s->n : 0};
    VQC_TRY(apply_single(s, m, qb, dm + 16, kind));
  }
  return VQC_OK;
}

static vqc_status apply_channel_dev(vqc_state s, int m, const int *q, int type, double prm,
                                    const std::vector<c128> &kraus_rm, int n_data) {
  c128 *dm = s->mat.as<c128>();
  c128 *kd = dm + 256;  // Kraus data scratch (up to 256 entries)
  if (!kraus_rm.empty()) {
    if (kraus_rm.size() > 256) {
      VQC_TRY(s->small.ensure(kraus_rm.size() * sizeof(c128)));
      kd = s->small.as<c128>();
    }
    VQC_TRY(hipMemcpyAsync(kd, kraus_rm.data(), kraus_rm.size() * sizeof(c128), hipMemcpyHostToDevice, s->stream));
    VQC_TRY(hipStreamSynchronize(s->stream));
  }
  if (m == 3) {  // Kraus sets only (validated): applied term by term, no 64 x 64 superoperator
    VQC_TRY(launch_kraus3(s->buf, s->nbits, s->n, q, kd, (int)(kraus_rm.size() / 64), s->stream));
    VQC_TRY(hipStreamSynchronize(s->stream));  // scratch reuse
    return VQC_OK;
  }
  DRecipe r;
  std::memset(&r, 0, sizeof(r));
  r.type = type;
  r.form = RF_SUPER_KRAUS;
  r.nq = m;
  r.data = kraus_rm.empty() ? -1 : 0;
  r.n_data = n_data;
  for (int k = 0; k < 5; k++) r.pidx[k] = -1;
  r.pval[0] = prm;
  VQC_TRY(launch_build_one(r, kraus_rm.empty() ? nullptr : kd, dm, s->stream));
  if (m == 1) {
    VQC_TRY(launch_g2(s->buf, s->nbits, q[0], q[0] + s->n, dm, SK_DENSE2, s->stream));
  } else {
    const int qq[4] = {q[0], q[1], q[0] + s->n, q[1] + s->n};
    VQC_TRY(launch_gm(s->buf, s->nbits, 4, qq, dm, s->stream));
  }
  if (!kraus_rm.empty()) VQC_TRY(hipStreamSynchronize(s->stream));  // scratch reuse
  return VQC_OK;
}

vqc_status vqc_apply_channel(vqc_state s, int m, const int *qubits, int n_kraus, const vqc_c128 *kraus) {
  if (!s || !qubits || !kraus || n_kraus < 1) return VQC_ERR_ARG;
  if (s->kind != VQC_MIXED) return VQC_ERR_KIND;
  if (m < 1 || m > 3) return VQC_ERR_UNSUPPORTED;
  vqc_op o;
  std::memset(&o, 0, sizeof(o));
  o.type = VQC_KRAUS;
  o.n_qubits = m;
  for (int i = 0; i < m; i++) o.qubits[i] = qubits[i];
  for (int k = 0; k < 5; k++) o.param_index[k] = -1;
  o.n_data = n_kraus * (1 << m) * (1 << m);
  o.data = kraus;
  return vqc_apply_op(s, &o);
}

static vqc_status expect_into(vqc_state s, const std::vector<DTerm> &terms, vqc_c128 *out) {
  const int iter_bits = s->n;  // pure: all amplitudes; mixed: the 2^n diagonal
  const int64_t units = expect_units(iter_bits);
  VQC_TRY(s->red.ensure(units * sizeof(double2) + 64));
  const size_t tb = std::max<size_t>(1, terms.size()) * sizeof(DTerm);
  VQC_TRY(s->small.ensure(tb + sizeof(DEJob) + 2 * sizeof(double2) + 512));
  char *sm = s->small.as<char>();
  DTerm *dterms = reinterpret_cast<DTerm *>(sm);
  DEJob *djob = reinterpret_cast<DEJob *>(sm + ((tb + 255) & ~size_t(255)));
  double2 *dres = reinterpret_cast<double2 *>(reinterpret_cast<char *>(djob) + 256);
  DEJob j;
  std::memset(&j, 0, sizeof(j));
  j.psi = s->buf;
  j.out = nullptr;
  j.partial = s->red.as<double2>();
  j.unit0 = 0;
  j.n_units = units;
  j.nbits = s->n;
  j.mixed = s->kind == VQC_MIXED;
  if (!terms.empty())
    VQC_TRY(hipMemcpyAsync(dterms, terms.data(), terms.size() * sizeof(DTerm), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(hipMemcpyAsync(djob, &j, sizeof(j), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(launch_expect(djob, 1, units, dterms, (int)terms.size(), s->stream));
  VQC_TRY(launch_reduce_partials(djob, 1, dres, s->stream));
  double2 r;
  VQC_TRY(hipMemcpyAsync(&r, dres, sizeof(r), hipMemcpyDeviceToHost, s->stream));
  VQC_TRY(hipStreamSynchronize(s->stream));
  out->re = r.x;
  out->im = r.y;
  return VQC_OK;
}

vqc_status vqc_expectation(vqc_state s, const vqc_pauli_sum *H, vqc_c128 *out) {
  if (!s || !H || !out) return VQC_ERR_ARG;
  std::vector<DTerm> terms;
  vqc_status st = make_terms(H, s->n, terms, false);
  if (st) return st;
  return expect_into(s, terms, out);
}

vqc_status vqc_expectation_noalloc(vqc_state s, const vqc_pauli_sum *H, vqc_c128 *out) {
  if (!s || !out || !pauli_sum_ok(H)) return VQC_ERR_ARG;
  const int64_t units = expect_units(s->n);
  if (H->n_terms > kNaMaxTerms || units > kNaMaxUnits) return VQC_ERR_SCRATCH_LIMIT;
  // terms staged in host memory that outlives the copy (the call ends with a
  // stream synchronisation); no heap allocation on this path
  DTerm terms[kNaMaxTerms];
  for (int t = 0; t < H->n_terms; t++) {
    const vqc_status st = make_term(H, t, s->n, false, terms[t]);
    if (st) return st;
  }
  char *sc = nullptr;
  VQC_TRY(na_scratch(s->stream, &sc));
  DTerm *dterms = reinterpret_cast<DTerm *>(sc + kNaTermOff);
  DEJob *djob = reinterpret_cast<DEJob *>(sc + kNaJobOff);
  double2 *dres = reinterpret_cast<double2 *>(sc + kNaResOff);
  DEJob j;
  std::memset(&j, 0, sizeof(j));
  j.psi = s->buf;
  j.out = nullptr;
  j.partial = reinterpret_cast<double2 *>(sc);  // every unit writes its own entry
  j.unit0 = 0;
  j.n_units = units;
  j.nbits = s->n;
  j.mixed = s->kind == VQC_MIXED;
  if (H->n_terms > 0)
    VQC_TRY(hipMemcpyAsync(dterms, terms, size_t(H->n_terms) * sizeof(DTerm), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(hipMemcpyAsync(djob, &j, sizeof(j), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(launch_expect(djob, 1, units, dterms, H->n_terms, s->stream));
  VQC_TRY(launch_reduce_partials(djob, 1, dres, s->stream));
  double2 r;
  VQC_TRY(hipMemcpyAsync(&r, dres, sizeof(r), hipMemcpyDeviceToHost, s->stream));
  VQC_TRY(hipStreamSynchronize(s->stream));
  out->re = r.x;
  out->im = r.y;
  return VQC_OK;
}

vqc_status vqc_norm(vqc_state s, double *out) {
  if (!s || !out) return VQC_ERR_ARG;
  std::vector<DTerm> terms(1);
  terms[0].xm = terms[0].zm = 0;
  terms[0].cre = 1.0;
  terms[0].cim = 0.0;
  vqc_c128 r;
  vqc_status st = expect_into(s, terms, &r);
  if (st) return st;
  *out = r.re;
  return VQC_OK;
}

vqc_status vqc_gather(vqc_state s, int count, const int64_t *idx, vqc_c128 *out) {
  if (!s || count < 0 || (count > 0 && (!idx || !out))) return VQC_ERR_ARG;
  if (s->kind != VQC_PURE) return VQC_ERR_KIND;
  if (count == 0) return VQC_OK;
  const int64_t N = int64_t(1) << s->n;
  for (int i = 0; i < count; i++)
    if (idx[i] < 0 || idx[i] >= N) return VQC_ERR_ARG;
  VQC_TRY(s->small.ensure(count * (sizeof(int64_t) + sizeof(c128)) + 256));
  int64_t *di = s->small.as<int64_t>();
  c128 *dout = reinterpret_cast<c128 *>(reinterpret_cast<char *>(di) + ((count * sizeof(int64_t) + 255) & ~size_t(255)));
  VQC_TRY(hipMemcpyAsync(di, idx, count * sizeof(int64_t), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(launch_gather(s->buf, di, count, dout, s->stream));
  VQC_TRY(hipMemcpyAsync(out, dout, count * sizeof(c128), hipMemcpyDeviceToHost, s->stream));
  VQC_TRY(hipStreamSynchronize(s->stream));
  return VQC_OK;
}

vqc_status vqc_measure(vqc_state s, int qubit, double u, int *outcome, double *prob) {
  if (!s || !outcome || !prob) return VQC_ERR_ARG;
  if (qubit < 0 || qubit >= s->n) return VQC_ERR_QUBIT;
  if (!is_finite_d(u)) return VQC_ERR_NONFINITE;
  if (u < 0.0 || u >= 1.0) return VQC_ERR_ARG;
  const int mixed = s->kind == VQC_MIXED;
  const int64_t m = prob_chunks(s->n);
  VQC_TRY(s->red.ensure((size_t)(m + 1) * sizeof(double2) + 256));
  double2 *part = s->red.as<double2>();
  double2 *res = part + m;
  VQC_TRY(launch_bit_mass(s->buf, s->n, mixed, qubit, part, res, s->stream));
  double2 h;
  VQC_TRY(hipMemcpyAsync(&h, res, sizeof(h), hipMemcpyDeviceToHost, s->stream));
  VQC_TRY(hipStreamSynchronize(s->stream));
  const double tot = h.x + h.y;
  if (!is_finite_d(tot)) return VQC_ERR_NONFINITE;
  if (!(tot > 0.0)) return VQC_ERR_ARG;
  const int o = u < h.x / tot ? 0 : 1;
  const double so = o ? h.y : h.x;
  *outcome = o;
  *prob = so / tot;
  const double scale = mixed ? 1.0 / so : 1.0 / std::sqrt(so);
  VQC_TRY(launch_collapse(s->buf, state_len(s->kind, s->n), s->n, mixed, qubit, o, scale, s->stream));
  return VQC_OK;
}

vqc_status vqc_sample(vqc_state s, int count, const double *u, int64_t *out) {
  if (!s || count < 0 || (count > 0 && (!u || !out))) return VQC_ERR_ARG;
  for (int k = 0; k < count; k++) {
    if (!is_finite_d(u[k])) return VQC_ERR_NONFINITE;
    if (u[k] < 0.0 || u[k] >= 1.0) return VQC_ERR_ARG;
  }
  const int mixed = s->kind == VQC_MIXED;
  const int64_t m = prob_chunks(s->n);
  const size_t cn = (size_t)std::max(1, count);
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  // mass | pref | cnt (2m) | off | u | out | chunk | perm | rem
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += al(bytes);
    return at;
  };
  const size_t o_mass = take(m * sizeof(double)), o_pref = take(m * sizeof(double));
  const size_t o_cnt = take(2 * m * sizeof(uint32_t)), o_off = take(m * sizeof(uint32_t));
  const size_t o_u = take(cn * sizeof(double)), o_out = take(cn * sizeof(int64_t));
  const size_t o_chunk = take(cn * sizeof(int32_t)), o_perm = take(cn * sizeof(int32_t));
  const size_t o_rem = take(cn * sizeof(double));
  VQC_TRY(s->red.ensure(o));
  char *base = s->red.as<char>();
  SampleBufs sb;
  sb.mass = reinterpret_cast<double *>(base + o_mass);
  sb.pref = reinterpret_cast<double *>(base + o_pref);
  sb.cnt = reinterpret_cast<uint32_t *>(base + o_cnt);
  sb.off = reinterpret_cast<uint32_t *>(base + o_off);
  sb.chunk = reinterpret_cast<int32_t *>(base + o_chunk);
  sb.perm = reinterpret_cast<int32_t *>(base + o_perm);
  sb.rem = reinterpret_cast<double *>(base + o_rem);
  double *du = reinterpret_cast<double *>(base + o_u);
  int64_t *dout = reinterpret_cast<int64_t *>(base + o_out);
  if (count > 0) VQC_TRY(hipMemcpyAsync(du, u, count * sizeof(double), hipMemcpyHostToDevice, s->stream));
  VQC_TRY(launch_sample(s->buf, s->n, mixed, sb, du, count, dout, s->stream));
  double total = 0.0;
  VQC_TRY(hipMemcpyAsync(&total, sb.pref + (m - 1), sizeof(double), hipMemcpyDeviceToHost, s->stream));
  if (count > 0) VQC_TRY(hipMemcpyAsync(out, dout, count * sizeof(int64_t), hipMemcpyDeviceToHost, s->stream));
  VQC_TRY(hipStreamSynchronize(s->stream));
  if (!is_finite_d(total)) return VQC_ERR_NONFINITE;
  if (!(total > 0.0)) return VQC_ERR_ARG;
  return VQC_OK;
}

// fuse_gates (Sec. 2.3): every op's matrix at theta, built on the device by
// the same recipes the circuits use, then the absorption on the host
vqc_status vqc_fuse_gates(int n, int n_ops, const vqc_op *ops, int n_params, const double *theta_host,
                          vqc_op *out_ops, vqc_c128 *out_data, int *n_out) {
  if (n < 1 || n > 33 || n_ops < 0 || !n_out || (n_ops > 0 && (!ops || !out_ops || !out_data))) return VQC_ERR_ARG;
  if (n_params < 0 || (n_params > 0 && !theta_host)) return VQC_ERR_ARG;
  for (int p = 0; p < n_params; p++)
    if (!is_finite_d(theta_host[p])) return VQC_ERR_NONFINITE;
  *n_out = 0;
  if (n_ops == 0) return VQC_OK;
  std::vector<DRecipe> rec(n_ops);
  std::vector<c128> cdata;
  for (int j = 0; j < n_ops; j++) {
    const vqc_op &op = ops[j];
    vqc_status st = validate_op(op, n, VQC_MIXED, n_params);
    if (st) return st;
    if (is_channel(op.type)) return VQC_ERR_KIND;  // noiseless circuits only
    if (op.n_qubits > 2) return VQC_ERR_UNSUPPORTED;
    DRecipe &r = rec[j];
    std::memset(&r, 0, sizeof(r));
    r.type = op.type;
    r.form = RF_GATE;
    r.nq = op.n_qubits;
    r.out = 16 * j;
    r.data = -1;
    if (op.data && op.n_data > 0) {
      r.data = (int)cdata.size();
      r.n_data = op.n_data;
      to_row_major(op.data, op.type == VQC_CONTROL ? 2 : 1 << op.n_qubits, cdata);
    }
    for (int k = 0; k < 5; k++) {
      r.pidx[k] = op.param_index[k];
      r.pval[k] = op.params[k];
    }
  }
  DevBuf drec, dcd, dth, dm;
  VQC_TRY(drec.ensure(rec.size() * sizeof(DRecipe)));
  VQC_TRY(dcd.ensure(std::max<size_t>(1, cdata.size()) * sizeof(c128)));
  VQC_TRY(dth.ensure(std::max(1, n_params) * sizeof(double)));
  VQC_TRY(dm.ensure((size_t)16 * n_ops * sizeof(c128)));
  VQC_TRY(hipMemcpy(drec.p, rec.data(), rec.size() * sizeof(DRecipe), hipMemcpyHostToDevice));
  if (!cdata.empty()) VQC_TRY(hipMemcpy(dcd.p, cdata.data(), cdata.size() * sizeof(c128), hipMemcpyHostToDevice));
  if (n_params > 0) VQC_TRY(hipMemcpy(dth.p, theta_host, n_params * sizeof(double), hipMemcpyHostToDevice));
  VQC_TRY(launch_build_mats(drec.as<DRecipe>(), n_ops, dcd.as<c128>(), nullptr, nullptr, 1, dth.as<double>(),
                            dm.as<c128>(), nullptr));
  std::vector<c128> M((size_t)16 * n_ops);
  VQC_TRY(hipMemcpy(M.data(), dm.p, M.size() * sizeof(c128), hipMemcpyDeviceToHost));
  // row-major d x d products; local bit t of a two-qubit op is its qubits[t]
  auto cm = [](c128 a, c128 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
  auto embed = [](const c128 *g, int t, c128 *G4) {  // g on local bit t of a 4x4
    for (int r = 0; r < 4; r++)
      for (int c = 0; c < 4; c++) {
        const int o = t ? 1 : 2;  // the other bit
        const bool same = ((r & o) != 0) == ((c & o) != 0);
        const int gr = (r >> t) & 1, gc = (c >> t) & 1;
        G4[r * 4 + c] = same ? g[gr * 2 + gc] : make_double2(0.0, 0.0);
      }
  };
  auto mul4 = [&](const c128 *A, const c128 *B, c128 *C) {
    for (int r = 0; r < 4; r++)
      for (int c = 0; c < 4; c++) {
        c128 acc = make_double2(0.0, 0.0);
        for (int k = 0; k < 4; k++) {
          const c128 p = cm(A[r * 4 + k], B[k * 4 + c]);
          acc.x += p.x;
          acc.y += p.y;
        }
        C[r * 4 + c] = acc;
      }
  };
  struct F {
    int m, q[2];
    c128 M[16];
  };
  std::vector<F> out;
  std::vector<int> last(n, -1);
  // applied until no one-qubit op sits next to a two-qubit op on its qubit:
  // a run of one-qubit ops goes into the two-qubit op before it (U <- g U),
  // else waits for the next two-qubit op on that qubit (U <- U g' ... g)
  std::vector<std::vector<int>> pending(n_ops);
  std::vector<int> next_two(n, -1), next2(n_ops, -1);
  for (int j = n_ops - 1; j >= 0; j--) {
    const vqc_op &op = ops[j];
    if (op.n_qubits == 1) next2[j] = next_two[op.qubits[0]];
    else
      for (int t = 0; t < op.n_qubits; t++) next_two[op.qubits[t]] = j;
  }
  for (int j = 0; j < n_ops; j++) {
    const vqc_op &op = ops[j];
    const c128 *G = M.data() + 16 * j;
    if (op.n_qubits == 1) {
      const int i = op.qubits[0], k = last[i];
      if (k >= 0 && out[k].m == 2) {  // right after a two-qubit op on i: U <- g U
        c128 G4[16], T[16];
        embed(G, out[k].q[0] == i ? 0 : 1, G4);
        mul4(G4, out[k].M, T);
        std::memcpy(out[k].M, T, sizeof(T));
      } else if (next2[j] >= 0) {  // right before one: U <- U g when it comes
        pending[next2[j]].push_back(j);
      } else {
        F f;
        f.m = 1;
        f.q[0] = i;
        f.q[1] = -1;
        std::memcpy(f.M, G, 4 * sizeof(c128));
        out.push_back(f);
        last[i] = (int)out.size() - 1;
      }
    } else {
      F f;
      f.m = 2;
      f.q[0] = op.qubits[0];
      f.q[1] = op.qubits[1];
      std::memcpy(f.M, G, 16 * sizeof(c128));
      for (int a = (int)pending[j].size() - 1; a >= 0; a--) {  // latest first: U g_last ... g_first
        const int pj = pending[j][a];
        c128 G4[16], T[16];
        embed(M.data() + 16 * pj, ops[pj].qubits[0] == f.q[0] ? 0 : 1, G4);
        mul4(f.M, G4, T);
        std::memcpy(f.M, T, sizeof(T));
      }
      out.push_back(f);
      last[f.q[0]] = last[f.q[1]] = (int)out.size() - 1;
    }
  }
  for (size_t k = 0; k < out.size(); k++) {
    const F &f = out[k];
    const int d = 1 << f.m;
    vqc_op &o = out_ops[k];
    std::memset(&o, 0, sizeof(o));
    o.type = VQC_MATRIX;
    o.n_qubits = f.m;
    o.qubits[0] = f.q[0];
    if (f.m == 2) o.qubits[1] = f.q[1];
    for (int p = 0; p < 5; p++) o.param_index[p] = -1;
    vqc_c128 *dst = out_data + 16 * k;
    for (int r = 0; r < d; r++)
      for (int c = 0; c < d; c++) {
        dst[r + d * c].re = f.M[r * d + c].x;  // column-major in the ABI
        dst[r + d * c].im = f.M[r * d + c].y;
      }
    o.data = dst;
    o.n_data = d * d;
  }
  *n_out = (int)out.size();
  return VQC_OK;
}

// -------------------------------------------------------------- circuits

namespace {

vqc_op plain_op(int type, int q0, int q1 = -1, const vqc_c128 *data = nullptr, int n_data = 0) {
  vqc_op o;
  std::memset(&o, 0, sizeof(o));
  o.type = type;
  o.n_qubits = q1 >= 0 ? 2 : 1;
  o.qubits[0] = q0;
  if (q1 >= 0) o.qubits[1] = q1;
  for (int k = 0; k < 5; k++) o.param_index[k] = -1;
  o.data = data;
  o.n_data = n_data;
  return o;
}

// T^dagger = diag(1, e^{-i pi/4}), column-major
const vqc_c128 kTdg[4] = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.70710678118654752440, -0.70710678118654752440}};

// Toffoli (controls a, b; target t) as six CNOTs with H, T and T^dagger
// (Nielsen and Chuang, Fig. 4.9)
void expand_toffoli(int a, int b, int t, std::vector<vqc_op> &out) {
  out.push_back(plain_op(VQC_H, t));
  out.push_back(plain_op(VQC_CNOT, b, t));
  out.push_back(plain_op(VQC_MATRIX, t, -1, kTdg, 4));
  out.push_back(plain_op(VQC_CNOT, a, t));
  out.push_back(plain_op(VQC_T, t));
  out.push_back(plain_op(VQC_CNOT, b, t));
  out.push_back(plain_op(VQC_MATRIX, t, -1, kTdg, 4));
  out.push_back(plain_op(VQC_CNOT, a, t));
  out.push_back(plain_op(VQC_T, b));
  out.push_back(plain_op(VQC_T, t));
  out.push_back(plain_op(VQC_H, t));
  out.push_back(plain_op(VQC_CNOT, a, b));
  out.push_back(plain_op(VQC_T, a));
  out.push_back(plain_op(VQC_MATRIX, b, -1, kTdg, 4));
  out.push_back(plain_op(VQC_CNOT, a, b));
}

// a three-qubit gate as exact one- and two-qubit ops; matrices it needs are
// kept in `store` (stable addresses)
vqc_status expand_gate3(const vqc_op &op, std::vector<vqc_op> &out, std::deque<std::vector<vqc_c128>> &store) {
  const int a = op.qubits[0], b = op.qubits[1], t = op.qubits[2];
  if (op.type == VQC_TOFFOLI) {
    expand_toffoli(a, b, t, out);
  } else if (op.type == VQC_FREDKIN) {  // CNOT(t->b) . Toffoli(a, b; t) . CNOT(t->b)
    out.push_back(plain_op(VQC_CNOT, t, b));
    expand_toffoli(a, b, t, out);
    out.push_back(plain_op(VQC_CNOT, t, b));
  } else if (op.type == VQC_CCONTROL) {
    // CV(b,t) CNOT(a,b) CV^dagger(b,t) CNOT(a,b) CV(a,t), V^2 = U
    // (Barenco et al. 1995, Lemma 6.1); V = (U + s I) / sqrt(tr U + 2 s),
    // s = sqrt(det U) with the sign that keeps the denominator away from 0
    using cd = std::complex<double>;
    const vqc_c128 *u = op.data;  // column-major: u[out + 2 in]
    c128 rm[4] = {make_double2(u[0].re, u[0].im), make_double2(u[2].re, u[2].im), make_double2(u[1].re, u[1].im),
                  make_double2(u[3].re, u[3].im)};
    if (!unitary_rm(rm, 2)) return VQC_ERR_NOT_UNITARY;
    const cd u00(u[0].re, u[0].im), u10(u[1].re, u[1].im), u01(u[2].re, u[2].im), u11(u[3].re, u[3].im);
    const cd tr = u00 + u11;
    cd sd = std::sqrt(u00 * u11 - u01 * u10);
    if (std::abs(tr - 2.0 * sd) > std::abs(tr + 2.0 * sd)) sd = -sd;
    const cd den = std::sqrt(tr + 2.0 * sd);
    const cd v[4] = {(u00 + sd) / den, u10 / den, u01 / den, (u11 + sd) / den};  // column-major
    store.emplace_back(4);
    std::vector<vqc_c128> &V = store.back();
    store.emplace_back(4);
    std::vector<vqc_c128> &Vd = store.back();
    for (int i = 0; i < 4; i++) V[i] = {v[i].real(), v[i].imag()};
    for (int r = 0; r < 2; r++)
      for (int c = 0; c < 2; c++) {  // (V^dagger)[r][c] = conj(V[c][r])
        const cd x = std::conj(v[c + 2 * r]);
        Vd[r + 2 * c] = {x.real(), x.imag()};
      }
    out.push_back(plain_op(VQC_CONTROL, b, t, V.data(), 4));
    out.push_back(plain_op(VQC_CNOT, a, b));
    out.push_back(plain_op(VQC_CONTROL, b, t, Vd.data(), 4));
    out.push_back(plain_op(VQC_CNOT, a, b));
    out.push_back(plain_op(VQC_CONTROL, a, t, V.data(), 4));
  } else if (op.type == VQC_MATRIX) {
    out.push_back(op);  // a register op on three bits (GK_DENSE3)
  } else {
    return VQC_ERR_UNSUPPORTED;  // three-qubit Kraus sets: single ops only
  }
  return VQC_OK;
}

}  // namespace

vqc_status vqc_circuit_create(vqc_circuit *out, int n, vqc_kind kind, int n_ops, const vqc_op *ops, int n_params,
                              const vqc_tune *tune) {
  if (!out || n_ops < 0 || (n_ops > 0 && !ops) || n_params < 0) return VQC_ERR_ARG;
  if (kind != VQC_PURE && kind != VQC_MIXED) return VQC_ERR_ARG;
  if (n < 1 || (kind == VQC_PURE && n > 33) || (kind == VQC_MIXED && n > 16)) return VQC_ERR_ARG;
  if (tune && (tune->tile_bits < 0 || tune->tile_bits > kMaxTile || tune->low_bits < 0 || tune->grid_blocks < 0 ||
               (tune->reg_bits != 0 && tune->reg_bits != 3 && tune->reg_bits != 4) || tune->remap < -1 ||
               tune->remap > 1 || tune->jit < -1 || tune->jit > 1))
    return VQC_ERR_ARG;
  for (int j = 0; j < n_ops; j++) {
    vqc_status st = validate_op(ops[j], n, kind, n_params);
    if (st) return st;
  }
  std::unique_ptr<vqc_circuit_s> c(new (std::nothrow) vqc_circuit_s());
  if (!c) return VQC_ERR_OOM;
  c->n = n;
  c->kind = kind;
  c->nbits = kind == VQC_MIXED ? 2 * n : n;
  c->n_params = n_params;
  std::memset(&c->tune, 0, sizeof(c->tune));
  if (tune) c->tune = *tune;
  std::deque<std::vector<vqc_c128>> store;  // matrices of expanded ops, alive through lowering
  for (int j = 0; j < n_ops; j++) {
    if (ops[j].n_qubits == 3 && ops[j].type != VQC_KRAUS) {
      vqc_status st = expand_gate3(ops[j], c->ops, store);
      if (st) return st;
    } else {
      c->ops.push_back(ops[j]);
    }
  }
  vqc_status st = lower(c.get());
  for (auto &o : c->ops) o.data = nullptr;  // data copied into cdata
  if (st) return st;
  st = make_plans(c.get());
  if (st) return st;
  st = upload_const(c.get());
  if (st) return st;
  st = jit_prepare(c.get());
  if (st) return st;
  *out = c.release();
  return VQC_OK;
}

vqc_status vqc_circuit_destroy(vqc_circuit c) {
  if (c && c->live_batches > 0) return VQC_ERR_IN_USE;
  delete c;
  return VQC_OK;
}

vqc_status vqc_circuit_stats_get(vqc_circuit c, vqc_circuit_stats *out) {
  if (!c || !out) return VQC_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->n_ops = (int)c->ops.size();
  out->n_elementary = (int)c->elems.size();
  out->n_passes = (int)c->fwd.passes.size();
  out->n_stages = c->fwd.n_stages;
  out->n_var = c->n_gslots;
  out->n_params = c->n_params;
  out->tune = c->tune;
  // algorithmic bytes per amplitude of the unfused ops (reads + writes of the
  // amplitudes each op must touch): dense 32 B, phase on |1> 16 B, CZ 8 B,
  // CNOT 16 B, fSim 24 B
  double b = 0;
  for (const Elem &e : c->elems) {
    switch (e.kind) {
      case GK_DIAG2: b += 32; break;
      case GK_CX: b += 16; break;
      case GK_FSIM: b += 24; break;
      case GK_NONE: break;
      default: b += 32; break;
    }
  }
  out->alg_bytes_per_amp = b;
  out->n_adj_passes = (int)c->adj.passes.size();
  for (const PassH &ph : c->fwd.passes) out->n_fwd_moves += ph.moves;
  for (const PassH &ph : c->adj.passes) out->n_adj_moves += ph.moves;
  out->n_jit_passes = c->fwd.jit ? (int)c->fwd.passes.size() : 0;
  out->n_jit_adj_passes = c->adj.jit ? (int)c->adj.passes.size() : 0;
  out->jit_ms = c->jit_ms;
  out->jit_cached = c->jit_cached ? 1 : 0;
  return VQC_OK;
}

vqc_status vqc_apply_circuit(vqc_state s, vqc_circuit c, const double *theta) {
  if (!s || !c) return VQC_ERR_ARG;
  if (s->kind != c->kind || s->n != c->n) return VQC_ERR_KIND;
  if (c->n_params > 0 && !theta) return VQC_ERR_ARG;
  c128 *mats = c->mats1.as<c128>();
  VQC_TRY(build_mats(c, nullptr, nullptr, 1, theta, mats, s->stream));
  VQC_TRY(run_passes(c, c->fwd, 0, s->buf, nullptr, mats, nullptr, 0, (int)c->fwd.passes.size(), 1, s->stream));
  return VQC_OK;
}

vqc_status vqc_apply_circuit_out(vqc_state dst, const vqc_state src, vqc_circuit c, const double *theta) {
  if (!dst || !src || !c) return VQC_ERR_ARG;
  if (src->kind != dst->kind || src->n != dst->n) return VQC_ERR_KIND;
  if (dst->buf == src->buf) return vqc_apply_circuit(dst, c, theta);
  VQC_TRY(launch_copy(dst->buf, src->buf, state_len(dst->kind, dst->n), dst->stream));
  return vqc_apply_circuit(dst, c, theta);
}

vqc_status vqc_apply_circuit_timed(vqc_state s, vqc_circuit c, const double *theta, float *pass_ms) {
  if (!s || !c || !pass_ms) return VQC_ERR_ARG;
  if (s->kind != c->kind || s->n != c->n) return VQC_ERR_KIND;
  if (c->n_params > 0 && !theta) return VQC_ERR_ARG;
  const int np = (int)c->fwd.passes.size();
  std::vector<hipEvent_t> ev(np + 1);
  for (auto &e : ev) VQC_TRY(hipEventCreate(&e));
  c128 *mats = c->mats1.as<c128>();
  hipError_t err = build_mats(c, nullptr, nullptr, 1, theta, mats, s->stream);
  if (err == hipSuccess) err = hipEventRecord(ev[0], s->stream);
  for (int p = 0; p < np && err == hipSuccess; p++) {
    err = run_passes(c, c->fwd, 0, s->buf, nullptr, mats, nullptr, p, p + 1, 1, s->stream);
    if (err == hipSuccess) err = hipEventRecord(ev[p + 1], s->stream);
  }
  if (err == hipSuccess) err = hipEventSynchronize(ev[np]);
  for (int p = 0; p < np && err == hipSuccess; p++) err = hipEventElapsedTime(&pass_ms[p], ev[p], ev[p + 1]);
  for (auto &e : ev) (void)hipEventDestroy(e);
  return hip_status(err);
}

static vqc_status seed_and_energy(vqc_circuit c, const std::vector<DTerm> &terms, const c128 *psi, c128 *out,
                                  hipStream_t st, double2 **res) {
  // expectation (and H psi when out != nullptr) of one item
  const int64_t units = expect_units(c->n);
  const size_t tb = ((std::max<size_t>(1, terms.size()) * sizeof(DTerm)) + 255) & ~size_t(255);
  VQC_TRY(c->ework.ensure(units * sizeof(double2) + tb + 1024));
  char *base = c->ework.as<char>();
  double2 *part = reinterpret_cast<double2 *>(base);
  char *rest = base + ((units * sizeof(double2) + 255) & ~size_t(255));
  DTerm *dterms = reinterpret_cast<DTerm *>(rest);
  DEJob *djob = reinterpret_cast<DEJob *>(rest + tb);
  double2 *dres = reinterpret_cast<double2 *>(rest + tb + 256);
  DEJob j;
  std::memset(&j, 0, sizeof(j));
  j.psi = psi;
  j.out = out;
  j.partial = part;
  j.n_units = units;
  j.nbits = c->n;
  j.mixed = c->kind == VQC_MIXED;
  if (!terms.empty())
    VQC_TRY(hipMemcpyAsync(dterms, terms.data(), terms.size() * sizeof(DTerm), hipMemcpyHostToDevice, st));
  VQC_TRY(hipMemcpyAsync(djob, &j, sizeof(j), hipMemcpyHostToDevice, st));
  VQC_TRY(hipStreamSynchronize(st));  // host sources above are locals
  VQC_TRY(launch_expect(djob, 1, units, dterms, (int)terms.size(), st));
  VQC_TRY(launch_reduce_partials(djob, 1, dres, st));
  *res = dres;
  return VQC_OK;
}

// energy_dev: optional device destination of the energy (stream-ordered);
// max_cond > 0 selects the inverse form for mixed circuits
static vqc_status backward_impl(vqc_circuit c, const double *theta, vqc_state s, const vqc_pauli_sum *H,
                                double *grad, double *energy_host, double *energy_dev, const void *init_dev,
                                size_t budget, double max_cond = 0.0) {
  if (!c || !s || !H) return VQC_ERR_ARG;
  if (s->kind != c->kind || s->n != c->n) return VQC_ERR_KIND;
  if (c->n_params > 0 && (!theta || !grad)) return VQC_ERR_ARG;
  std::vector<DTerm> terms;
  vqc_status vs = make_terms(H, c->n, terms, true);
  if (vs) return vs;
  hipStream_t st = s->stream;
  const uint64_t N = state_len(c->kind, c->n);
  c128 *mats = c->mats1.as<c128>();
  Plan &P = c->adj;
  Plan *PG = &P;  // the plan whose partials hold the gradient
  const int np = (int)P.passes.size();
  VQC_TRY(c->part1.ensure(std::max<size_t>(1, (size_t)c->n_gslots) * P.units_per_item * sizeof(double) + 256));
  double2 *dres = nullptr;
  if (c->kind == VQC_PURE) {
    if (c->has_nonunitary_matrix) return VQC_ERR_NOT_UNITARY;
    VQC_TRY(c->psi1.ensure(N * sizeof(c128)));
    if (P.needs_scratch && c->scratch2.ensure(N * sizeof(c128)) != hipSuccess) return VQC_ERR_OOM;
    c128 *psi = c->psi1.as<c128>();
    VQC_TRY(build_mats(c, nullptr, nullptr, 1, theta, mats, st));
    vs = seed_and_energy(c, terms, s->buf, psi, st, &dres);
    if (vs) return vs;
    VQC_TRY(run_passes(c, P, 1, s->buf, psi, mats, c->part1.as<double>(), 0, np, -1, st));
  } else if (max_cond > 0.0) {
    // inverse form: invert the non-unitary ops' matrices, check their
    // condition numbers, then one sweep with Phi <- M^{-1} Phi
    if (c->has_nonunitary_matrix) return VQC_ERR_NOT_UNITARY;
    VQC_TRY(c->psi1.ensure(N * sizeof(c128)));
    c128 *psi = c->psi1.as<c128>();
    VQC_TRY(build_mats(c, nullptr, nullptr, 1, theta, mats, st));
    if (c->n_special && !(c->special_kappa <= max_cond)) return VQC_ERR_ILL_CONDITIONED;
    if (!c->inv_list.empty()) {
      unsigned long long *kb = c->dinv.as<unsigned long long>();
      VQC_TRY(hipMemsetAsync(kb, 0, sizeof(*kb), st));
      VQC_TRY(launch_invert(reinterpret_cast<const DInv *>(c->dinv.as<char>() + 256), (int)c->inv_list.size(),
                            nullptr, 1, mats, kb, st));
      unsigned long long bits = 0;
      VQC_TRY(hipMemcpyAsync(&bits, kb, sizeof(bits), hipMemcpyDeviceToHost, st));
      VQC_TRY(hipStreamSynchronize(st));
      double kappa;
      std::memcpy(&kappa, &bits, sizeof(kappa));
      if (!(kappa <= max_cond)) return VQC_ERR_ILL_CONDITIONED;
    }
    std::vector<DTerm> tt = terms;
    VQC_TRY(c->small.ensure(std::max<size_t>(1, tt.size()) * sizeof(DTerm)));
    if (!tt.empty())
      VQC_TRY(hipMemcpyAsync(c->small.p, tt.data(), tt.size() * sizeof(DTerm), hipMemcpyHostToDevice, st));
    VQC_TRY(hipStreamSynchronize(st));
    VQC_TRY(launch_seed_mixed(psi, c->n, c->small.as<DTerm>(), (int)tt.size(), st));
    vs = seed_and_energy(c, terms, s->buf, nullptr, st, &dres);
    if (vs) return vs;
    Plan &PI = inv_adj(c);
    PG = &PI;
    VQC_TRY(c->part1.ensure(std::max<size_t>(1, (size_t)c->n_gslots) * PI.units_per_item * sizeof(double) + 256));
    if (PI.needs_scratch && c->scratch2.ensure(N * sizeof(c128)) != hipSuccess) return VQC_ERR_OOM;
    // register-only plans take the inverse-form mode; LDS plans apply M^{-1}
    // for the ops flagged non-unitary in their adjoint step
    VQC_TRY(run_passes(c, PI, PI.reg_only ? 3 : 1, s->buf, psi, mats, c->part1.as<double>(), 0,
                       (int)PI.passes.size(), -1, st));
  } else {
    // checkpoints every `stride` passes; a segment of states is recomputed
    // from its checkpoint before its backward steps
    const size_t SB = N * sizeof(c128);
    size_t bud = budget ? budget : (size_t)16 << 30;
    int best = -1;
    size_t best_need = 0;
    for (int sd = 1; sd <= std::max(1, np); sd++) {
      const size_t need = (size_t)((np + sd - 1) / sd + (sd - 1) + 2) * SB;
      if (need <= bud && (best < 0 || need < best_need)) { best = sd; best_need = need; }
    }
    if (best < 0) return VQC_ERR_OOM;
    const int sd = best;
    const int nck = (np + sd - 1) / sd;
    VQC_TRY(c->ck.ensure(best_need));
    c128 *W = c->ck.as<c128>();
    c128 *psi = W + N;
    c128 *ck0 = psi + N;
    c128 *seg0 = ck0 + (size_t)nck * N;
    VQC_TRY(build_mats(c, nullptr, nullptr, 1, theta, mats, st));
    if (init_dev) VQC_TRY(launch_copy(W, reinterpret_cast<const c128 *>(init_dev), N, st));
    else VQC_TRY(launch_init_basis0(W, N, st));
    Plan &F = ck_fwd(c);
    for (int p = 0; p < np; p++) {
      if (p % sd == 0) VQC_TRY(launch_copy(ck0 + (size_t)(p / sd) * N, W, N, st));
      VQC_TRY(run_passes(c, F, 0, W, nullptr, mats, nullptr, p, p + 1, 1, st));
    }
    {
      // vec(H) needs the terms on device
      std::vector<DTerm> tt = terms;
      VQC_TRY(c->small.ensure(std::max<size_t>(1, tt.size()) * sizeof(DTerm)));
      if (!tt.empty())
        VQC_TRY(hipMemcpyAsync(c->small.p, tt.data(), tt.size() * sizeof(DTerm), hipMemcpyHostToDevice, st));
      VQC_TRY(hipStreamSynchronize(st));
      VQC_TRY(launch_seed_mixed(psi, c->n, c->small.as<DTerm>(), (int)tt.size(), st));
    }
    vs = seed_and_energy(c, terms, W, nullptr, st, &dres);
    if (vs) return vs;
    for (int k = nck - 1; k >= 0; k--) {
      const int s0 = k * sd, s1 = std::min(np, s0 + sd);
      auto segp = [&](int i) { return i == 0 ? ck0 + (size_t)k * N : seg0 + (size_t)(i - 1) * N; };
      for (int i = 1; i < s1 - s0; i++)
        VQC_TRY(run_passes(c, F, 0, segp(i - 1), segp(i), mats, nullptr, s0 + i - 1, s0 + i, 1, st));
      for (int p = s1 - 1; p >= s0; p--)
        VQC_TRY(run_passes(c, P, 2, segp(p - s0), psi, mats, c->part1.as<double>(), p, p + 1, 1, st));
    }
  }
  if (c->n_params > 0) {
    DGradJob gj;
    gj.partials = c->part1.as<double>();
    gj.n_units = PG->units_per_item;
    gj.grad = grad;
    gj.csr_ptr = c->d_csr_ptr;
    gj.csr_slot = c->d_csr_slot;
    gj.n_params = c->n_params;
    gj.scale = c->kind == VQC_PURE ? 2.0 : 1.0;
    VQC_TRY(c->small.ensure(sizeof(DGradJob) + 256));
    DGradJob *dg = reinterpret_cast<DGradJob *>(c->small.as<char>());
    VQC_TRY(hipMemcpyAsync(dg, &gj, sizeof(gj), hipMemcpyHostToDevice, st));
    VQC_TRY(hipStreamSynchronize(st));
    VQC_TRY(launch_grad_reduce(dg, 1, c->n_params, st));
  }
  if (energy_dev) VQC_TRY(launch_take_real(dres, 1, energy_dev, st));
  if (energy_host) {
    double2 r;
    VQC_TRY(hipMemcpyAsync(&r, dres, sizeof(r), hipMemcpyDeviceToHost, st));
    VQC_TRY(hipStreamSynchronize(st));
    *energy_host = r.x;
  }
  return VQC_OK;
}

vqc_status vqc_backward(vqc_circuit c, const double *theta, vqc_state s, const vqc_pauli_sum *H, double *grad,
                        double *energy_host, const void *init_dev, size_t budget) {
  return backward_impl(c, theta, s, H, grad, energy_host, nullptr, init_dev, budget);
}

vqc_status vqc_backward_inverse(vqc_circuit c, const double *theta, vqc_state s, const vqc_pauli_sum *H,
                                double *grad, double *energy_host, double max_cond) {
  if (!c) return VQC_ERR_ARG;
  if (!is_finite_d(max_cond)) return VQC_ERR_NONFINITE;
  if (c->kind == VQC_PURE) return backward_impl(c, theta, s, H, grad, energy_host, nullptr, nullptr, 0);
  return backward_impl(c, theta, s, H, grad, energy_host, nullptr, nullptr, 0, max_cond > 0.0 ? max_cond : 1e8);
}

// one timed run of an autotune candidate: forward (target 0) or forward +
// gradient (target 1) from |0..0>, on the scratch state s
static vqc_status tune_run(vqc_circuit c, vqc_state s, const double *theta, const vqc_pauli_sum *H, int target,
                           double *grad) {
  vqc_status st = vqc_state_reset(s);
  if (st) return st;
  st = vqc_apply_circuit(s, c, theta);
  if (st || target == 0) return st;
  return backward_impl(c, theta, s, H, grad, nullptr, nullptr, nullptr, 0);
}

vqc_status vqc_circuit_autotune_ex(vqc_circuit c, vqc_state s, const double *theta, const vqc_pauli_sum *H,
                                   int target, vqc_tune *out) {
  if (!c || !s || !out || (target != VQC_TUNE_FORWARD && target != VQC_TUNE_GRADIENT)) return VQC_ERR_ARG;
  if (s->kind != c->kind || s->n != c->n) return VQC_ERR_KIND;
  if (c->n_params > 0 && !theta) return VQC_ERR_ARG;
  if (target == VQC_TUNE_GRADIENT && !H) return VQC_ERR_ARG;
  // a batch holds device pointers into the circuit's plans: re-planning would
  // leave them dangling
  if (c->live_batches > 0) return VQC_ERR_IN_USE;
  const bool mixed = c->kind == VQC_MIXED;
  if ((mixed && c->nbits < kMixedLdsMinBits) || c->nbits < 5) {  // register-only plans: nothing to choose
    *out = c->tune;
    return VQC_OK;
  }
  if (target == VQC_TUNE_GRADIENT) {
    std::vector<DTerm> t;
    const vqc_status st = make_terms(H, c->n, t, true);
    if (st) return st;
  }
  DevBuf gbuf;
  double *grad = nullptr;
  if (target == VQC_TUNE_GRADIENT) {
    VQC_TRY(gbuf.ensure(std::max(1, c->n_params) * sizeof(double)));
    grad = gbuf.as<double>();
  }
  // candidates: tile and low-block bits, register bits; qubit moves on and
  // off at the default shape (mixed: low-block bits and qubit moves)
  const vqc_tune orig = c->tune;
  std::vector<vqc_tune> cand;
  auto add = [&](int K, int low, int R, int remap) {
    vqc_tune t = orig;
    t.tile_bits = K;
    t.low_bits = low;
    t.reg_bits = R;
    t.remap = remap;
    for (const vqc_tune &u : cand)
      if (u.tile_bits == K && u.low_bits == low && u.reg_bits == R && u.remap == remap) return;
    cand.push_back(t);
  };
  if (mixed) {
    for (int low = 3; low <= 6; low++) add(kMixedTile, low, 4, orig.remap);
    add(kMixedTile, orig.low_bits, 4, orig.remap > 0 ? -1 : 1);
  } else {
    add(orig.tile_bits, orig.low_bits, orig.reg_bits, orig.remap);
    for (int K = std::min(11, c->nbits); K >= std::max(8, std::min(10, c->nbits)); K--)
      for (int low = 3; low <= 5; low++)
        for (int R = 3; R <= 4; R++)
          if (low <= K - 2) add(K, low, R, orig.remap);
    if (c->nbits >= kRemapMinBits) add(orig.tile_bits, orig.low_bits, orig.reg_bits, orig.remap > 0 ? -1 : 1);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_status(he);
  }
  vqc_tune best = orig;
  float best_ms = 3.0e38f;
  for (const vqc_tune &t : cand) {
    c->tune = t;
    if (make_plans(c) != VQC_OK || jit_prepare(c, target == VQC_TUNE_GRADIENT) != VQC_OK) continue;
    // warm-up, then enough repetitions for a few milliseconds of work
    if (tune_run(c, s, theta, H, target, grad) != VQC_OK) continue;
    if (hipStreamSynchronize(s->stream) != hipSuccess) continue;
    int reps = 1;
    float ms = 0;
    bool ok = true;
    for (;;) {
      ok = hipEventRecord(e0, s->stream) == hipSuccess;
      for (int r = 0; ok && r < reps; r++) ok = tune_run(c, s, theta, H, target, grad) == VQC_OK;
      ok = ok && hipEventRecord(e1, s->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (!ok || ms >= 20.0f || reps >= 64) break;
      reps *= 4;
    }
    if (!ok) continue;
    ms /= reps;
    if (ms < best_ms) {
      best_ms = ms;
      best = c->tune;  // as resolved by the planner
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tune = best_ms < 3.0e38f ? best : orig;
  vqc_status st = make_plans(c);
  if (st == VQC_OK) st = upload_const(c);
  if (st == VQC_OK) st = jit_prepare(c, true);
  if (st) return st;
  if (best_ms >= 3.0e38f) return VQC_ERR_HIP;  // no candidate ran
  *out = c->tune;
  return VQC_OK;
}

vqc_status vqc_circuit_autotune(vqc_circuit c, vqc_state s, const double *theta, vqc_tune *out) {
  return vqc_circuit_autotune_ex(c, s, theta, nullptr, VQC_TUNE_FORWARD, out);
}

// --------------------------------------------------------------- batches

static vqc_status batch_build_tables(vqc_batch b) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const int B = b->B;
  // per-item matrices, Psi, partials, expectation partials
  size_t mtot = 0, ptot = 0, qtot = 0;
  int64_t etot = 0;
  b->mat_off.resize(B);
  b->psi_off.resize(B);
  b->part_off.resize(B);
  std::vector<int64_t> e_off(B);
  for (int i = 0; i < B; i++) {
    vqc_circuit c = b->circ[i];
    b->mat_off[i] = mtot;
    mtot += al((size_t)c->mat_total * sizeof(c128));
    b->psi_off[i] = ptot;
    ptot += al(state_len(c->kind, c->n) * sizeof(c128));  // allocated by the backward
    b->part_off[i] = qtot;
    qtot += al(std::max(1, c->n_gslots) * batch_adj(c).units_per_item * sizeof(double));
    e_off[i] = etot;
    etot += expect_units(c->n);
    b->max_passes = std::max(b->max_passes, (int)c->fwd.passes.size());
    b->max_adj = std::max(b->max_adj, (int)batch_adj(c).passes.size());
    b->max_params = std::max(b->max_params, c->n_params);
  }
  b->e_units = etot;
  VQC_TRY(b->mats.ensure(mtot));
  // scratch states: one for the forward, two for the adjoint once Psi exists
  size_t stot = 0;
  b->scr_off.assign(B, 0);
  for (int i = 0; i < B; i++) {
    vqc_circuit c = b->circ[i];
    b->scr_off[i] = stot;
    const size_t sb = al(state_len(c->kind, c->n) * sizeof(c128));
    const bool adj = b->psi.p && batch_adj(c).needs_scratch;
    if (c->fwd.needs_scratch || adj) stot += sb;
    if (adj) stot += sb;
  }
  if (stot) VQC_TRY(b->scr.ensure(stot));
  auto scr_state = [&](int i, int k) {
    const size_t sb = al(state_len(b->circ[i]->kind, b->circ[i]->n) * sizeof(c128));
    return reinterpret_cast<c128 *>(b->scr.as<char>() + b->scr_off[i] + k * sb);
  };
  VQC_TRY(b->eparts.ensure(etot * sizeof(double2) + al(B * sizeof(double2)) + 256));
  b->d_eres = reinterpret_cast<double2 *>(b->eparts.as<char>() + al(etot * sizeof(double2)));
  // groups of items sharing a circuit: pointer arrays for the matrix build
  std::vector<vqc_circuit> uniq;
  for (int i = 0; i < B; i++)
    if (std::find(uniq.begin(), uniq.end(), b->circ[i]) == uniq.end()) uniq.push_back(b->circ[i]);
  for (vqc_circuit c : uniq) {
    std::unique_ptr<vqc_batch_s::Group> g(new vqc_batch_s::Group());
    g->c = c;
    std::vector<const void *> ptrs;
    std::vector<const void *> th, mt;
    for (int i = 0; i < B; i++)
      if (b->circ[i] == c) {
        th.push_back(b->thetas[i]);
        mt.push_back(b->mats.as<char>() + b->mat_off[i]);
      }
    g->count = (int)th.size();
    ptrs.insert(ptrs.end(), th.begin(), th.end());
    ptrs.insert(ptrs.end(), mt.begin(), mt.end());
    VQC_TRY(g->ptrs.ensure(ptrs.size() * sizeof(void *)));
    VQC_TRY(hipMemcpy(g->ptrs.p, ptrs.data(), ptrs.size() * sizeof(void *), hipMemcpyHostToDevice));
    b->groups.push_back(std::move(g));
  }
  // forward step jobs
  std::vector<DJob> fj;
  for (int sI = 0; sI < b->max_passes; sI++) {
    b->fwd_first.push_back((int)fj.size());
    int64_t u0 = 0;
    for (int i = 0; i < B; i++) {
      vqc_circuit c = b->circ[i];
      if (sI >= (int)c->fwd.passes.size()) continue;
      DJob j;
      std::memset(&j, 0, sizeof(j));
      j.a = b->states[i];
      if (c->fwd.needs_scratch) {
        c128 *bufs[2] = {b->states[i], scr_state(i, 0)};
        const PassH &ph = c->fwd.passes[sI];
        j.a = bufs[ph.src];
        j.b = bufs[ph.dst];
        j.mode = ph.src != ph.dst ? 1 : 0;
      }
      j.mats = reinterpret_cast<const c128 *>(b->mats.as<char>() + b->mat_off[i]);
      j.pass = c->fwd.d_pass + sI;
      j.unit0 = u0;
      j.n_units = c->fwd.units_per_item;
      j.nbits = c->nbits;
      u0 += j.n_units;
      fj.push_back(j);
    }
    b->fwd_count.push_back((int)fj.size() - b->fwd_first.back());
    b->fwd_units.push_back(u0);
  }
  // adjoint step jobs (aligned at each item's last pass; pure: Alg. 2, mixed:
  // its inverse form)
  std::vector<DJob> aj;
  for (int r = 0; r < b->max_adj; r++) {
    b->adj_first.push_back((int)aj.size());
    int64_t u0 = 0;
    for (int i = 0; i < B; i++) {
      vqc_circuit c = b->circ[i];
      const Plan &A = batch_adj(c);
      const int PA = (int)A.passes.size();
      if (r >= PA) continue;
      DJob j;
      std::memset(&j, 0, sizeof(j));
      j.a = b->states[i];
      j.b = reinterpret_cast<c128 *>(b->psi.p ? b->psi.as<char>() + b->psi_off[i] : nullptr);
      j.mats = reinterpret_cast<const c128 *>(b->mats.as<char>() + b->mat_off[i]);
      j.partials = reinterpret_cast<double *>(b->part.p ? b->part.as<char>() + b->part_off[i] : nullptr);
      if (b->psi.p && A.needs_scratch) {
        // reverse order: read the pass's destination, write its source
        c128 *bufs[2] = {j.a, scr_state(i, 0)}, *bufb[2] = {j.b, scr_state(i, 1)};
        const PassH &ph = A.passes[PA - 1 - r];
        j.a = bufs[ph.dst];
        j.b = bufb[ph.dst];
        j.a2 = bufs[ph.src];
        j.b2 = bufb[ph.src];
        j.mode = ph.src != ph.dst ? 1 : 0;
      }
      j.pass = A.d_pass + (PA - 1 - r);
      j.unit0 = u0;
      j.n_units = A.units_per_item;
      j.nbits = c->nbits;
      u0 += j.n_units;
      aj.push_back(j);
    }
    b->adj_count.push_back((int)aj.size() - b->adj_first.back());
    b->adj_units.push_back(u0);
  }
  // expectation and seed jobs
  std::vector<DEJob> ej(B), sj(B);
  for (int i = 0; i < B; i++) {
    vqc_circuit c = b->circ[i];
    DEJob &e = ej[i];
    std::memset(&e, 0, sizeof(e));
    e.psi = b->states[i];
    e.partial = b->eparts.as<double2>() + e_off[i];
    e.unit0 = e_off[i];
    e.n_units = expect_units(c->n);
    e.nbits = c->n;
    e.mixed = c->kind == VQC_MIXED;
    sj[i] = e;
    if (c->kind == VQC_PURE && b->psi.p) sj[i].out = reinterpret_cast<c128 *>(b->psi.as<char>() + b->psi_off[i]);
  }
  std::vector<c128 *> sp(b->states);
  std::vector<uint64_t> sz(B);
  uint64_t maxn = 0;
  for (int i = 0; i < B; i++) {
    sz[i] = state_len(b->circ[i]->kind, b->circ[i]->n);
    maxn = std::max(maxn, sz[i]);
  }
  (void)maxn;
  const size_t o_f = 0, o_a = al(o_f + fj.size() * sizeof(DJob)), o_e = al(o_a + aj.size() * sizeof(DJob));
  const size_t o_s = al(o_e + B * sizeof(DEJob)), o_p = al(o_s + B * sizeof(DEJob));
  const size_t o_z = al(o_p + B * sizeof(c128 *)), o_g = al(o_z + B * sizeof(uint64_t));
  const size_t total = al(o_g + B * sizeof(DGradJob));
  VQC_TRY(b->tables.ensure(total));
  std::vector<char> blob(total, 0);
  std::memcpy(blob.data() + o_f, fj.data(), fj.size() * sizeof(DJob));
  std::memcpy(blob.data() + o_a, aj.data(), aj.size() * sizeof(DJob));
  std::memcpy(blob.data() + o_e, ej.data(), B * sizeof(DEJob));
  std::memcpy(blob.data() + o_s, sj.data(), B * sizeof(DEJob));
  std::memcpy(blob.data() + o_p, sp.data(), B * sizeof(c128 *));
  std::memcpy(blob.data() + o_z, sz.data(), B * sizeof(uint64_t));
  char *base = b->tables.as<char>();
  VQC_TRY(hipMemcpy(base, blob.data(), total, hipMemcpyHostToDevice));
  b->d_fwd_jobs = reinterpret_cast<DJob *>(base + o_f);
  b->d_adj_jobs = reinterpret_cast<DJob *>(base + o_a);
  b->d_ejobs = reinterpret_cast<DEJob *>(base + o_e);
  b->d_sjobs = reinterpret_cast<DEJob *>(base + o_s);
  b->d_state_ptrs = reinterpret_cast<c128 **>(base + o_p);
  b->d_state_sizes = reinterpret_cast<uint64_t *>(base + o_z);
  b->d_gjobs = reinterpret_cast<DGradJob *>(base + o_g);
  return VQC_OK;
}

static vqc_status batch_forward_on(vqc_batch b, hipStream_t st) {
  uint64_t maxn = 0;
  for (int i = 0; i < b->B; i++) maxn = std::max(maxn, state_len(b->circ[i]->kind, b->circ[i]->n));
  VQC_TRY(launch_init_batched(b->d_state_ptrs, b->d_state_sizes, b->B, maxn, st));
  for (auto &g : b->groups) {
    const double *const *th = reinterpret_cast<const double *const *>(g->ptrs.p);
    c128 *const *mt = reinterpret_cast<c128 *const *>(g->ptrs.as<char>() + g->count * sizeof(void *));
    VQC_TRY(build_mats(g->c, th, mt, g->count, nullptr, nullptr, st));
  }
  DOverride ov;
  std::memset(&ov, 0, sizeof(ov));
  vqc_circuit c0 = b->circ[0];
  // every item runs the same circuit: step sI is that circuit's pass sI
  bool same = true;
  for (int i = 1; i < b->B; i++) same = same && b->circ[i] == c0;
  for (int sI = 0; sI < b->max_passes; sI++) {
    const int64_t units = b->fwd_units[sI];
    const int grid = grid_of(c0, units);
    const DJob *jobs = b->d_fwd_jobs + b->fwd_first[sI];
    ov.job_units = same ? c0->fwd.units_per_item : 0;
    if (same && c0->fwd.jit) VQC_TRY(launch_jit_pass(*c0->fwd.jit, sI, c0->fwd, jobs, b->fwd_count[sI], units, ov, st));
    else if (b->reg_only) VQC_TRY(launch_pass_reg(c0->fwd.R, 0, jobs, b->fwd_count[sI], units, grid, ov, st));
    else VQC_TRY(launch_pass_lds(c0->fwd.K, c0->fwd.R, false, c0->fwd.d4, jobs, b->fwd_count[sI], units, grid, ov,
                                 st));
  }
  return VQC_OK;
}

static vqc_status batch_upload_terms(vqc_batch b, const vqc_pauli_sum *H, bool need_real) {
  int nmax = 0;
  for (int i = 0; i < b->B; i++) nmax = std::max(nmax, b->circ[i]->n);
  int nmin = 64;
  for (int i = 0; i < b->B; i++) nmin = std::min(nmin, b->circ[i]->n);
  std::vector<DTerm> t;
  vqc_status st = make_terms(H, nmin, t, need_real);
  if (st) return st;
  b->terms_h = t;
  b->n_terms = (int)t.size();
  VQC_TRY(b->ck.ensure(std::max<size_t>(1, t.size()) * sizeof(DTerm)));  // ck doubles as term storage
  b->d_terms = b->ck.as<DTerm>();
  if (!t.empty()) VQC_TRY(hipMemcpy(b->d_terms, t.data(), t.size() * sizeof(DTerm), hipMemcpyHostToDevice));
  return VQC_OK;
}

static vqc_status batch_ensure_adjoint(vqc_batch b) {
  if (b->psi.p) return VQC_OK;
  size_t ptot = 0, qtot = 0;
  for (int i = 0; i < b->B; i++) {
    vqc_circuit c = b->circ[i];
    ptot = std::max(ptot, b->psi_off[i] + ((state_len(c->kind, c->n) * sizeof(c128) + 255) & ~size_t(255)));
    qtot = std::max(qtot, b->part_off[i] + ((std::max(1, c->n_gslots) * batch_adj(c).units_per_item * sizeof(double) + 255) &
                                            ~size_t(255)));
  }
  VQC_TRY(b->psi.ensure(std::max<size_t>(ptot, 16)));
  VQC_TRY(b->part.ensure(std::max<size_t>(qtot, 16)));
  // rebuild tables now that Psi / partials exist
  b->groups.clear();
  b->fwd_first.clear(); b->fwd_count.clear(); b->fwd_units.clear();
  b->adj_first.clear(); b->adj_count.clear(); b->adj_units.clear();
  b->max_passes = b->max_adj = b->max_params = 0;
  return batch_build_tables(b);
}

static vqc_status batch_grad_jobs(vqc_batch b, double *const *grads, bool mixed_inverse = false) {
  std::vector<DGradJob> gj(b->B);
  for (int i = 0; i < b->B; i++) {
    vqc_circuit c = b->circ[i];
    DGradJob &g = gj[i];
    std::memset(&g, 0, sizeof(g));
    g.partials = reinterpret_cast<const double *>(b->part.as<char>() + b->part_off[i]);
    g.n_units = batch_adj(c).units_per_item;
    g.grad = grads[i];
    g.csr_ptr = c->d_csr_ptr;
    g.csr_slot = c->d_csr_slot;
    g.n_params = (c->kind == VQC_PURE || mixed_inverse) ? c->n_params : 0;
    g.scale = c->kind == VQC_PURE ? 2.0 : 1.0;
  }
  VQC_TRY(hipMemcpy(b->d_gjobs, gj.data(), gj.size() * sizeof(DGradJob), hipMemcpyHostToDevice));
  return VQC_OK;
}

// pure items: seed, reverse passes, gradient reduction; energies optional
static vqc_status batch_backward_pure_on(vqc_batch b, double *energies, hipStream_t st) {
  for (auto &g : b->groups) {
    const double *const *th = reinterpret_cast<const double *const *>(g->ptrs.p);
    c128 *const *mt = reinterpret_cast<c128 *const *>(g->ptrs.as<char>() + g->count * sizeof(void *));
    VQC_TRY(build_mats(g->c, th, mt, g->count, nullptr, nullptr, st));
  }
  VQC_TRY(launch_expect(b->d_sjobs, b->B, b->e_units, b->d_terms, b->n_terms, st));
  VQC_TRY(launch_reduce_partials(b->d_sjobs, b->B, b->d_eres, st));
  if (energies) VQC_TRY(launch_take_real(b->d_eres, b->B, energies, st));
  DOverride ov;
  std::memset(&ov, 0, sizeof(ov));
  vqc_circuit c0 = b->circ[0];
  bool same = true;  // every item runs the same circuit: step r is its pass PA - 1 - r
  for (int i = 1; i < b->B; i++) same = same && b->circ[i] == c0;
  for (int r = 0; r < b->max_adj; r++) {
    if (b->adj_count[r] == 0) continue;
    const int64_t units = b->adj_units[r];
    const int grid = grid_of(c0, units);
    const DJob *jobs = b->d_adj_jobs + b->adj_first[r];
    const int PA = (int)c0->adj.passes.size();
    ov.job_units = same ? c0->adj.units_per_item : 0;
    if (same && c0->adj.jit && r < PA)
      VQC_TRY(launch_jit_pass(*c0->adj.jit, PA - 1 - r, c0->adj, jobs, b->adj_count[r], units, ov, st));
    else
      VQC_TRY(launch_pass_lds(c0->adj.K, c0->adj.R, true, false, jobs, b->adj_count[r], units, grid, ov, st));
  }
  VQC_TRY(launch_grad_reduce(b->d_gjobs, b->B, b->max_params, st));
  return VQC_OK;
}

vqc_status vqc_batch_create(vqc_batch *out, int B, const vqc_circuit *circuits, void *const *states,
                            const double *const *thetas, void *stream) {
  if (!out || B < 1 || !circuits || !states) return VQC_ERR_ARG;
  for (int i = 0; i < B; i++) {
    if (!circuits[i] || !states[i]) return VQC_ERR_ARG;
    if (circuits[i]->n_params > 0 && (!thetas || !thetas[i])) return VQC_ERR_ARG;
    const vqc_circuit c = circuits[i], c0 = circuits[0];
    if (c->kind != c0->kind) return VQC_ERR_KIND;
    if (c->n_special > 0) return VQC_ERR_UNSUPPORTED;  // three-qubit channels: single circuits only
    const Plan &A = batch_adj(c), &A0 = batch_adj(c0);
    if (c->fwd.reg_only != c0->fwd.reg_only || c->fwd.K != c0->fwd.K || c->fwd.R != c0->fwd.R ||
        c->fwd.d4 != c0->fwd.d4 || A.K != A0.K || A.R != A0.R || A.reg_only != A0.reg_only || A.d4 != A0.d4)
      return VQC_ERR_UNSUPPORTED;
  }
  std::unique_ptr<vqc_batch_s> b(new (std::nothrow) vqc_batch_s());
  if (!b) return VQC_ERR_OOM;
  b->B = B;
  b->circ.assign(circuits, circuits + B);
  for (int i = 0; i < B; i++) {
    b->states.push_back(reinterpret_cast<c128 *>(states[i]));
    b->thetas.push_back(thetas ? thetas[i] : nullptr);
  }
  b->stream = reinterpret_cast<hipStream_t>(stream);
  b->reg_only = circuits[0]->fwd.reg_only;
  b->K = circuits[0]->fwd.K;
  b->Kadj = circuits[0]->adj.K;
  vqc_status st = batch_build_tables(b.get());
  if (st) return st;
  for (vqc_circuit c : b->circ) c->live_batches++;
  *out = b.release();
  return VQC_OK;
}

vqc_status vqc_batch_destroy(vqc_batch b) {
  if (!b) return VQC_OK;
  for (vqc_circuit c : b->circ) c->live_batches--;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return VQC_OK;
}

vqc_status vqc_batch_forward(vqc_batch b) {
  if (!b) return VQC_ERR_ARG;
  return batch_forward_on(b, b->stream);
}

vqc_status vqc_batch_expectation(vqc_batch b, const vqc_pauli_sum *H, double *energies) {
  if (!b || !H || !energies) return VQC_ERR_ARG;
  VQC_TRY(hipStreamSynchronize(b->stream));
  vqc_status st = batch_upload_terms(b, H, false);
  if (st) return st;
  VQC_TRY(launch_expect(b->d_ejobs, b->B, b->e_units, b->d_terms, b->n_terms, b->stream));
  VQC_TRY(launch_reduce_partials(b->d_ejobs, b->B, b->d_eres, b->stream));
  VQC_TRY(launch_take_real(b->d_eres, b->B, energies, b->stream));
  return VQC_OK;
}

vqc_status vqc_batch_backward(vqc_batch b, const vqc_pauli_sum *H, double *const *grads, double *energies,
                              size_t budget) {
  if (!b || !H || !grads) return VQC_ERR_ARG;
  for (int i = 0; i < b->B; i++)
    if (b->circ[i]->n_params > 0 && !grads[i]) return VQC_ERR_ARG;
  VQC_TRY(hipStreamSynchronize(b->stream));
  if (b->circ[0]->kind == VQC_PURE) {
    for (int i = 0; i < b->B; i++)
      if (b->circ[i]->has_nonunitary_matrix) return VQC_ERR_NOT_UNITARY;
    vqc_status st = batch_ensure_adjoint(b);
    if (st) return st;
    st = batch_upload_terms(b, H, true);
    if (st) return st;
    st = batch_grad_jobs(b, grads);
    if (st) return st;
    return batch_backward_pure_on(b, energies, b->stream);
  }
  // mixed items: checkpointed backward item by item on the batch stream (the
  // sweep recomputes the forward from |0><0| itself; the items' states are
  // only read for their shape)
  for (int i = 0; i < b->B; i++) {
    vqc_state_s it;
    it.kind = VQC_MIXED;
    it.n = b->circ[i]->n;
    it.nbits = 2 * it.n;
    it.buf = b->states[i];
    it.stream = b->stream;
    vqc_status st = backward_impl(b->circ[i], b->thetas[i], &it, H, grads[i], nullptr,
                                  energies ? energies + i : nullptr, nullptr, budget);
    if (st) return st;
  }
  return VQC_OK;
}

// inverse form for a batch of mixed items: all items' passes step together
vqc_status vqc_batch_backward_inverse(vqc_batch b, const vqc_pauli_sum *H, double *const *grads, double *energies,
                                      double max_cond) {
  if (!b || !H || !grads) return VQC_ERR_ARG;
  if (!is_finite_d(max_cond)) return VQC_ERR_NONFINITE;
  if (b->circ[0]->kind == VQC_PURE) return vqc_batch_backward(b, H, grads, energies, 0);
  const double bound = max_cond > 0.0 ? max_cond : 1e8;
  for (int i = 0; i < b->B; i++) {
    if (b->circ[i]->n_params > 0 && !grads[i]) return VQC_ERR_ARG;
    if (b->circ[i]->has_nonunitary_matrix) return VQC_ERR_NOT_UNITARY;
  }
  VQC_TRY(hipStreamSynchronize(b->stream));
  vqc_status st = batch_ensure_adjoint(b);
  if (st) return st;
  st = batch_upload_terms(b, H, true);
  if (st) return st;
  st = batch_grad_jobs(b, grads, true);
  if (st) return st;
  hipStream_t s = b->stream;
  VQC_TRY(b->kappa.ensure(256));
  unsigned long long *kb = b->kappa.as<unsigned long long>();
  VQC_TRY(hipMemsetAsync(kb, 0, sizeof(*kb), s));
  for (auto &g : b->groups) {
    const double *const *th = reinterpret_cast<const double *const *>(g->ptrs.p);
    c128 *const *mt = reinterpret_cast<c128 *const *>(g->ptrs.as<char>() + g->count * sizeof(void *));
    VQC_TRY(build_mats(g->c, th, mt, g->count, nullptr, nullptr, s));
    if (!g->c->inv_list.empty())
      VQC_TRY(launch_invert(reinterpret_cast<const DInv *>(g->c->dinv.as<char>() + 256), (int)g->c->inv_list.size(),
                            mt, g->count, nullptr, kb, s));
  }
  unsigned long long bits = 0;
  VQC_TRY(hipMemcpyAsync(&bits, kb, sizeof(bits), hipMemcpyDeviceToHost, s));
  VQC_TRY(hipStreamSynchronize(s));
  double kappa;
  std::memcpy(&kappa, &bits, sizeof(kappa));
  if (!(kappa <= bound)) return VQC_ERR_ILL_CONDITIONED;
  for (int i = 0; i < b->B; i++)
    VQC_TRY(launch_seed_mixed(reinterpret_cast<c128 *>(b->psi.as<char>() + b->psi_off[i]), b->circ[i]->n, b->d_terms,
                              b->n_terms, s));
  VQC_TRY(launch_expect(b->d_ejobs, b->B, b->e_units, b->d_terms, b->n_terms, s));
  VQC_TRY(launch_reduce_partials(b->d_ejobs, b->B, b->d_eres, s));
  if (energies) VQC_TRY(launch_take_real(b->d_eres, b->B, energies, s));
  DOverride ov;
  std::memset(&ov, 0, sizeof(ov));
  vqc_circuit c0 = b->circ[0];
  for (int r = 0; r < b->max_adj; r++) {
    if (b->adj_count[r] == 0) continue;
    const int64_t units = b->adj_units[r];
    const int grid = grid_of(c0, units);
    const DJob *jobs = b->d_adj_jobs + b->adj_first[r];
    const Plan &A0 = inv_adj(c0);
    if (A0.reg_only) VQC_TRY(launch_pass_reg(A0.R, 3, jobs, b->adj_count[r], units, grid, ov, s));
    else VQC_TRY(launch_pass_lds(A0.K, A0.R, true, A0.d4, jobs, b->adj_count[r], units, grid, ov, s));
  }
  VQC_TRY(launch_grad_reduce(b->d_gjobs, b->B, b->max_params, s));
  return VQC_OK;
}

vqc_status vqc_batch_capture(vqc_batch b, const vqc_pauli_sum *H, double *const *grads, double *energies,
                             size_t budget) {
  (void)budget;
  if (!b || !H || !grads) return VQC_ERR_ARG;
  if (b->circ[0]->kind != VQC_PURE) return VQC_ERR_UNSUPPORTED;
  for (int i = 0; i < b->B; i++)
    if (b->circ[i]->n_params > 0 && !grads[i]) return VQC_ERR_ARG;
  VQC_TRY(hipStreamSynchronize(b->stream));
  vqc_status st = batch_ensure_adjoint(b);
  if (st) return st;
  st = batch_upload_terms(b, H, true);
  if (st) return st;
  st = batch_grad_jobs(b, grads);
  if (st) return st;
  if (b->gexec) { (void)hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  if (!b->cap_stream) VQC_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  // one eager run so that every kernel attribute is set before capture
  st = batch_forward_on(b, b->cap_stream);
  if (!st) st = batch_backward_pure_on(b, energies, b->cap_stream);
  if (st) return st;
  VQC_TRY(hipStreamSynchronize(b->cap_stream));
  VQC_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  vqc_status s1 = batch_forward_on(b, b->cap_stream);
  vqc_status s2 = s1 ? s1 : batch_backward_pure_on(b, energies, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (s2) { if (g) (void)hipGraphDestroy(g); return s2; }
  if (e != hipSuccess) return hip_status(e);
  b->graph = g;
  VQC_TRY(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
  return VQC_OK;
}

vqc_status vqc_batch_replay(vqc_batch b) {
  if (!b || !b->gexec) return VQC_ERR_ARG;
  VQC_TRY(hipGraphLaunch(b->gexec, b->stream));
  return VQC_OK;
}

}  // extern "C"

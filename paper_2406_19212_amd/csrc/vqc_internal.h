// Internal tables shared by the host planner (api.cpp) and the gfx950
// kernels (kernels.hip).  Not part of the C ABI.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#else
// compiled at run time (hipRTC) for circuit-specialised pass kernels: the
// fixed-width integer types are declared in a namespace there
using __hip_internal::int8_t;
using __hip_internal::int16_t;
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint8_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace vqc {

typedef double2 c128;  // (re, im)

// Register-level kinds of an elementary op (a gate, a half of a gate acting on
// the ket or bra bits of vec(rho), or a superoperator).
enum GateKind : int8_t {
  GK_DENSE1 = 0,  // 2x2 on one bit
  GK_DIAG1 = 1,   // diag(m00, m11)
  GK_DENSE2 = 2,  // 4x4 on two bits (local index b0 + 2 b1)
  GK_DIAG2 = 3,   // diag(m00, m11, m22, m33)
  GK_FSIM = 4,    // m00 | [[m11 m12][m21 m22]] | m33 (fSim / iSWAP pattern)
  GK_CX = 5,      // controlled X: control bit 0, target bit 1 (no matrix)
  GK_DENSE4 = 6,  // 16x16 on four bits, register bits 0..3 in order
  GK_NONE = 7,    // identity (no-op)
  GK_XROT1 = 8,   // [[a, i b], [i c, d]], a..d real (Rx, phase-free sqrt(X), Y)
  GK_REAL1 = 9,   // real 2x2 (Ry, H, X, phase-free sqrt(Y))
  GK_RDIAG1 = 10, // real diagonal, complex off-diagonal (phase-free sqrt(W))
  GK_FSIMX = 11,  // fSim with Delta = 0: 1 | [[c, -i s], [-i s, c]] | e^{-i phi}
  GK_PHASE1 = 12, // diag(1, m11)
  // in-place rotation forms: the op's matrix is followed by an SRec whose
  // plane rotations are applied as three shears each (u += a v; v += b u;
  // u += a v), so every update is an accumulate into the amplitude's own
  // register.  g.mat of these kinds points at the SRec.
  GK_SXR1 = 13,   // [[c, -i s], [-i s, c]] (Rx, phase-free sqrt(X))
  GK_SRR1 = 14,   // [[c, -s], [s, c]] (Ry, phase-free sqrt(Y))
  GK_SPH1 = 15,   // diag(1, e^{i p}) (Z, S, T)
  GK_SDG1 = 16,   // diag(e^{i p0}, e^{i p1}) (Rz, global phase)
  GK_SRD1 = 17,   // D^dagger R D, D = diag(1, e^{i chi}) (phase-free sqrt(W))
  GK_SFX = 18,    // fSim with Delta = 0 as two rotations of the |01>,|10> block and one phase
  // derivative-only kinds of U = exp(-i theta G / 2), G = X, Y, Z on one bit:
  // Re<Psi| dU |Phi_before> = Im<Psi| G |Phi_after> / 2, evaluated before
  // Phi is uncomputed through U (no derivative matrix)
  GK_GENX = 19,
  GK_GENY = 20,
  GK_GENZ = 21,
  // a two-qubit depolarizing superoperator a I + b |I>><<I| on (q1, q2,
  // q1 + n, q2 + n), register bits 0..3 in order: a = M[1][1], b = M[0][5]
  // of its stored 16x16 (the inverse has the same form)
  GK_DEPOL4 = 22,
  // 8x8 on three register bits (a general three-qubit gate; local index
  // b_{q0} + 2 b_{q1} + 4 b_{q2})
  GK_DENSE3 = 23,
  // a three-qubit channel on vec(rho) (6 bits): not a register op; the
  // planner gives it a pass of its own, run by k_kraus3
  GK_KRAUS3 = 24,
  // sqrt(X), sqrt(Y), sqrt(W) (phase-factored) times sqrt(2), for the
  // specialised forward passes: four additions per pair for the first two,
  // four additions and four FMAs for the third; the pass multiplies its tile
  // by 2^(-k/2) for its k such ops before storing it
  GK_HX1 = 25,    // [[1, -i], [-i, 1]]
  GK_HY1 = 26,    // [[1, -1], [1, 1]]
  GK_HW1 = 27     // [[1, e^{-3 i pi/4}], [e^{-i pi/4}, 1]]
};
// DGate.nd: derivative count in the low byte; this bit set when the op's
// derivatives are generator kinds (taken on Phi before the op is undone)
constexpr int kGenFlag = 0x100;
// DGate.nd: the op is not unitary (a channel, or a fused run holding one);
// its inverse superoperator is stored right after its matrix
constexpr int kInvFlag = 0x200;

// Shear record of a rotation kind.  Rotation i by angle p (cos p = C,
// sin p = S) is stored as a = -S/(1+C), b = S with C >= 0; an angle with
// C < 0 is stored as the rotation by p - pi and bit i of neg set (the
// rotation then ends with both coordinates negated).
struct SRec {
  uint32_t neg;
  uint32_t pad;
  double ab[7];     // (a, b) of rotations 0..2, one spare
};
static_assert(sizeof(SRec) == 64, "SRec is four c128 slots");
constexpr int kSRecSlots = 4;

constexpr int kMaxTile = 13;      // K <= 13: 2^13 * 16 B = 128 KiB of LDS
constexpr int kMaxVarPerPass = 256;  // derivative slots reduced inside one pass

// one elementary op inside a pass, in stage-local register bits
struct DGate {
  int8_t kind;
  int8_t nq;
  int8_t r[4];      // register bit of the op's local qubit t
  int16_t nd;       // derivative records (adjoint only)
  int32_t mat;      // matrix offset in the item's matrix buffer (c128 units), -1 none
  int32_t d0;       // first derivative record
};

// Op g of a plan as the pass kernels read it: the static descriptor plus the
// item's rotation record, stored in execution order inside the item's matrix
// buffer so that each op is one 64 B scalar load at an address known without
// reading anything else first.  Entry 0 and entry n+1 of a plan's program
// are padding (kind GK_NONE) so the kernels may read one op past either end
// of a stage.
struct DOp {
  DGate g;
  uint32_t neg;
  uint32_t pad;     // bit 31: one generator derivative, kind in bits 0-7, local slot in 8-23
  double ab[5];     // rotation parameters (GK_S* kinds), as in SRec
};
static_assert(sizeof(DOp) == 64, "DOp is four c128 slots");
constexpr int kOpSlots = 4;

struct DDeriv {
  int8_t kind;      // register kind of the derivative matrix
  int8_t pad[3];
  int32_t mat;      // derivative matrix offset (c128 units)
  int32_t gslot;    // global derivative slot (row of the partials array)
  int32_t local;    // slot inside the pass reduction (0 .. nvar-1)
};

struct DStage {
  int8_t rbit[4];   // tile-local bit held in register bit i
  int8_t srt[4];    // the same bits, sorted ascending (zero insertion)
  int32_t g0, g1;   // gate range [g0, g1) of this stage (absolute index)
};

struct DPass {
  int32_t K;        // tile bits (= R for register-only passes)
  int32_t nst;      // stages
  int32_t nvar;     // derivative slots reduced in this pass
  int32_t lowfree;  // bit 0: stage 0 holds none of the low c bits; bit 1: the last stage
                    // holds none (that stage can then load/store HBM directly, coalesced)
  int8_t tq[16];    // physical bit (input layout) of tile-local bit i, ascending
  int8_t tqo[16];   // output layout: physical bits of the tile, ascending ...
  int8_t lbo[16];   // ... and the tile-local bit stored at each (identity when the layout stays)
  int32_t prog;     // c128 offset of the plan's op program in the item's matrix buffer
  int32_t pad;
  const DStage *stages;   // absolute device pointers
  const DGate *gates;
  const DDeriv *derivs;
  const int32_t *vslot;   // gslot of pass-local derivative slot v
};

// a non-unitary op's matrix to invert (inverse-form noisy adjoint)
struct DInv {
  int32_t mat;  // matrix offset (c128 units); the inverse goes to mat + dim^2
  int32_t dim;  // 4 or 16
};

// one (item, pass) of a launch
struct DJob {
  c128 *a;          // state (forward) / Phi (adjoint)
  c128 *b;          // Psi (adjoint), or destination for out-of-place forward
  c128 *a2;         // out-of-place adjoint: destinations of Phi ...
  c128 *b2;         // ... and Psi
  const c128 *mats; // the item's matrices
  double *partials; // [gslot][n_units] (adjoint)
  const DPass *pass;
  int64_t unit0;    // first global unit of this job
  int64_t n_units;  // units (tiles, or blocks of tiles) of this job
  int32_t nbits;
  int32_t mode;     // 0: in place; 1: out of place (forward: read a, write b;
                    // adjoint: read a, b, write a2, b2)
};

// buffers for single-item launches, passed by value so that the device job
// tables stay static; use = 0 takes everything from the job
struct DOverride {
  c128 *a;
  c128 *b;
  c128 *a2;
  c128 *b2;
  const c128 *mats;
  double *partials;
  int32_t mode;
  int32_t use;
  // units of every job when all jobs of a launch have the same count (job j
  // holds units j * job_units ..): the job of a unit is a division instead
  // of a search; 0 = search (read by the circuit-specialised kernels)
  int64_t job_units;
};

// matrix recipes (built on device from theta)
enum RecipeForm : int32_t {
  RF_GATE = 0,      // gate matrix
  RF_GATE_CONJ = 1, // complex conjugate of the gate matrix (bra half)
  RF_DGATE = 2,     // derivative of the gate matrix w.r.t. parameter k
  RF_DGATE_CONJ = 3,
  RF_SUPER_GATE = 4,  // conj(U) (x) U  (ket bits low, bra bits high)
  RF_DSUPER_GATE = 5, // conj(dU) (x) U + conj(U) (x) dU
  RF_SUPER_KRAUS = 6,  // sum_s conj(K_s) (x) K_s
  RF_GATE_F = 7,       // gate matrix with the global phase e^{i pi/4} of sqrt(X/Y/W) removed
  RF_GPHASE = 8,       // diag(w, w), w = e^{i pi k / 4}
  // product S_{m-1} ... S_0 of the 4x4 superoperators of a run of one-qubit
  // ops (data = index of S_0's recipe in the recipe array, n_data = m)
  RF_FUSED = 9,
  RF_DFUSED = 10,      // the same with S_s replaced by its derivative: k = s * 8 + parameter
  RF_COPY = 11         // the op's constant matrix as stored (row-major), conjugated when k = 1
};

struct DRecipe {
  int32_t type;     // VQC_* op type
  int32_t form;
  int32_t k;        // parameter for derivatives
  int32_t nq;       // qubits of the original op
  int32_t out;      // output offset (c128 units)
  int32_t data;     // offset into the circuit's constant data (c128 units), -1 none
  int32_t n_data;   // entries at data
  int32_t pidx[5];  // theta index of each parameter, -1 = fixed
  int32_t shear;    // rotation kind whose SRec follows the matrix, 0 none
  int32_t pad;
  double pval[5];
};

struct DTerm {      // Pauli term with i^{|Y|} folded into the coefficient
  uint64_t xm, zm;
  double cre, cim;
};

struct DEJob {      // expectation / seed job (one item)
  const c128 *psi;
  c128 *out;        // H psi (pure seed) or vec(H) (mixed seed); nullptr if unused
  double2 *partial; // per-unit partial sums
  int64_t unit0, n_units;
  int32_t nbits;    // n (qubits, not vec bits)
  int32_t mixed;
};

struct DGradJob {
  const double *partials;  // [slot][n_units]
  int64_t n_units;
  double *grad;
  const int32_t *csr_ptr;  // parameter p -> slots [csr_ptr[p], csr_ptr[p+1])
  const int32_t *csr_slot;
  int32_t n_params;
  double scale;
};

// launchers (kernels.hip)
#ifndef __HIPCC_RTC__  // host launchers
hipError_t launch_pass_lds(int K, int R, bool adj, bool d4, const DJob *jobs, int n_jobs, int64_t total, int grid,
                           const DOverride &ov, hipStream_t st);
hipError_t launch_pass_reg(int R, int mode, const DJob *jobs, int n_jobs, int64_t total, int grid,
                           const DOverride &ov, hipStream_t st);
hipError_t launch_build_mats(const DRecipe *rec, int n_rec, const c128 *cdata, const double *const *thetas,
                             c128 *const *mats, int B, const double *theta0, c128 *mats0, hipStream_t st);
hipError_t launch_build_one(const DRecipe &r, const c128 *cdata, c128 *out, hipStream_t st);
hipError_t launch_assemble(const DGate *gates, const DDeriv *derivs, int n_gates, int prog, c128 *const *mats,
                           int B, c128 *mats0, hipStream_t st);
hipError_t launch_invert(const DInv *inv, int n_inv, c128 *const *mats, int B, c128 *mats0,
                         unsigned long long *kappa_bits, hipStream_t st);
hipError_t launch_init_batched(c128 *const *ptrs, const uint64_t *sizes, int B, uint64_t max_n, hipStream_t st);
int64_t expect_units(int nbits_iter);
hipError_t launch_expect(const DEJob *jobs, int n_jobs, int64_t total, const DTerm *terms, int nt, hipStream_t st);
hipError_t launch_reduce_partials(const DEJob *jobs, int n_jobs, double2 *out, hipStream_t st);
hipError_t launch_take_real(const double2 *in, int n, double *dst, hipStream_t st);
hipError_t launch_seed_mixed(c128 *out, int n, const DTerm *terms, int nt, hipStream_t st);
hipError_t launch_grad_reduce(const DGradJob *jobs, int n_items, int max_params, hipStream_t st);
hipError_t launch_g1(c128 *psi, int nbits, int q, const c128 *M, int kind, hipStream_t st);
hipError_t launch_g2(c128 *psi, int nbits, int q0, int q1, const c128 *M, int kind, hipStream_t st);
hipError_t launch_gm(c128 *psi, int nbits, int m, const int *q, const c128 *M, hipStream_t st);
hipError_t launch_kraus3(c128 *v, int nbits, int n, const int *q, const c128 *K, int nk, hipStream_t st);
// three-qubit channel on ket bits qk / bra bits qb (physical positions): the
// Kraus sum of nk matrices K (dense = 0) or a dense 64 x 64 superoperator K
hipError_t launch_block6(c128 *v, int nbits, const int *qk, const int *qb, const c128 *K, int nk, int dense,
                         hipStream_t st);
hipError_t launch_init_basis0(c128 *v, uint64_t N, hipStream_t st);
hipError_t launch_fill_zero(c128 *v, uint64_t N, hipStream_t st);
hipError_t launch_copy(c128 *dst, const c128 *src, uint64_t N, hipStream_t st);
hipError_t launch_gather(const c128 *psi, const int64_t *idx, int count, c128 *out, hipStream_t st);
int64_t prob_chunks(int n);  // blocks of basis states of the measurement / sampling kernels
hipError_t launch_bit_mass(const c128 *v, int n, int mixed, int q, double2 *part, double2 *out, hipStream_t st);
hipError_t launch_collapse(c128 *v, uint64_t len, int n, int mixed, int q, int outcome, double scale,
                           hipStream_t st);
// device buffers of one sampling call (m = prob_chunks(n) chunks, `count` samples)
struct SampleBufs {
  double *mass, *pref;   // [m] chunk masses and their running sums
  uint32_t *cnt;         // [2 m] samples per chunk, then the bucketing cursors
  uint32_t *off;         // [m] first bucket slot of each chunk
  int32_t *chunk, *perm; // [count] chunk of each sample; sample indices by chunk
  double *rem;           // [count] mass left to cover inside the chunk
};
hipError_t launch_sample(const c128 *v, int n, int mixed, const SampleBufs &sb, const double *u, int count,
                         int64_t *out, hipStream_t st);
hipError_t launch_set_mat(c128 *dst, const c128 *m, int count, hipStream_t st);

enum SingleKind { SK_DENSE1 = 0, SK_DIAG1, SK_PHASE1, SK_DENSE2, SK_DIAG2, SK_PHASE11, SK_FSIM, SK_CX, SK_CTRL };
constexpr int kEChunkHost = 4096;

#endif  // __HIPCC_RTC__
}  // namespace vqc

// Kernels of the surrogate network (energy landscape model, not part of the
// paper's method): C = op(A) op(B) with BF16 inputs rounded from FP32 and FP32
// accumulation on MFMA, the exact-erf GELU with its first and second
// derivatives, column sums for bias gradients, and Adam.  All FP32 storage.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <new>

#include "../../include/vqc.h"

namespace vqc {

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// FP32 -> BF16, round to nearest even: v_cvt_pk_bf16_f32 (two per instruction)
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
  const bf16x2v r = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, r);
}

// C[M x N] = alpha * op(A) op(B) + beta * C, op(A)[m][k] = A[m*lda + k] (ta = 0)
// or A[k*lda + m] (ta = 1); op(B)[k][n] = B[k*ldb + n] (tb = 0) or B[n*ldb + k].
//
// Block tile BT x BT (32, 64 or 128, chosen by the launcher so that the grid
// fills the chip), K step 64 or 128 (MFMA k blocks of 32), four waves in a 2 x 2
// arrangement, each owning a (BT/2) x (BT/2) quadrant of 16 x 16 MFMA tiles
// (v_mfma_f32_16x16x32_bf16: eight consecutive k per lane, the same k
// assignment for both operands, so each MFMA sums all 32 products of its k
// block).  The K loop is software
// pipelined: the FP32 slab of step k+1 is loaded into registers while step k
// runs from LDS, then rounded to BF16 into the other of two LDS buffers; one
// barrier per step.  Global loads follow the operand's contiguous dimension
// (float4 when the leading dimension and base are 16-byte aligned, otherwise
// four bounds-checked scalars), so every layout reads coalesced, and every
// layout stores 8-byte runs of k into LDS.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short s16x8;

// K step per tile: 128 for the 32 x 32 tile (small grids, where the number of
// dependent steps sets the time), 64 otherwise.  LDS rows are padded by 8
// (pitch 272 or 144 B): 16-byte aligned, and the 16 rows of an MFMA fragment
// read fall on distinct banks.
constexpr int kstep(int bt) { return bt == 32 ? 128 : 64; }

// one operand slab, BT rows (m for A, n for B) x GK k values, held in
// registers between the global load and the LDS store.  KC: the operand is
// contiguous along k (A with ta = 0, B with tb = 1); each thread moves float4
// groups of four consecutive k of one row.
template <int BT, bool KC>
struct Slab {
  static constexpr int GK = kstep(BT), GKP = GK + 8;
  static constexpr int NG = BT * GK / 4 / 256;  // float4 groups per thread
  float4 v[NG];

  __device__ __forceinline__ void load(const float *__restrict__ X, int ld, int rows, int K, int r0, int k0, bool vec,
                                       int t) {
#pragma unroll
    for (int i = 0; i < NG; i++) {
      const int q = t + 256 * i;
      const int gr = r0 + q / (GK / 4), gk = k0 + 4 * (q % (GK / 4));
      // (both branches fill e: assigning the float4 straight to v[i] made the
      // compiler split the vector load into a 12-byte and a 4-byte load)
      float e[4];
      if (vec && gr < rows && gk + 3 < K) {
        const float4 w = *(const float4 *)(X + (int64_t)gr * ld + gk);
        e[0] = w.x, e[1] = w.y, e[2] = w.z, e[3] = w.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; j++) e[j] = (gr < rows && gk + j < K) ? X[(int64_t)gr * ld + gk + j] : 0.f;
      }
      v[i] = make_float4(e[0], e[1], e[2], e[3]);
    }
  }

  // rounded to BF16 into Xs[row][k]
  __device__ __forceinline__ void store(short (*Xs)[GKP], int t) const {
#pragma unroll
    for (int i = 0; i < NG; i++) {
      const int q = t + 256 * i;
      *(uint2 *)&Xs[q / (GK / 4)][4 * (q % (GK / 4))] =
          make_uint2(bf16_pair(v[i].x, v[i].y), bf16_pair(v[i].z, v[i].w));
    }
  }
};

// Rows contiguous (A with ta = 1, B with tb = 0): each thread moves 4 x 4
// blocks (four float4 loads of four consecutive rows, at four consecutive k)
// and transposes them in registers, so that its LDS stores are 8-byte runs
// of k like the other layout's.  Eight consecutive threads take consecutive
// row groups (128 contiguous bytes per k), the next eight the next k group.
template <int BT>
struct Slab<BT, false> {
  static constexpr int GK = kstep(BT), GKP = GK + 8;
  static constexpr int RG = BT / 4, KG = GK / 4;    // 4 x 4 blocks per slab side
  static constexpr int NB = (RG * KG + 255) / 256;  // blocks per thread
  float v[NB][4][4];                                // [block][k][row]

  __device__ __forceinline__ static bool at(int q, int &rg, int &kg) {
    const int hi = q >> 3;
    kg = hi % KG;
    rg = (q & 7) + 8 * (hi / KG);
    return q < RG * KG;
  }

  __device__ __forceinline__ void load(const float *__restrict__ X, int ld, int rows, int K, int r0, int k0, bool vec,
                                       int t) {
#pragma unroll
    for (int b = 0; b < NB; b++) {
      int rg, kg;
      if (!at(t + 256 * b, rg, kg)) continue;
      const int gr = r0 + 4 * rg;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int gk = k0 + 4 * kg + j;
        float e[4];  // filled by both branches, which keeps the load one float4
        if (vec && gk < K && gr + 3 < rows) {
          const float4 w = *(const float4 *)(X + (int64_t)gk * ld + gr);
          e[0] = w.x, e[1] = w.y, e[2] = w.z, e[3] = w.w;
        } else {
#pragma unroll
          for (int r = 0; r < 4; r++) e[r] = (gk < K && gr + r < rows) ? X[(int64_t)gk * ld + gr + r] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < 4; r++) v[b][j][r] = e[r];
      }
    }
  }

  __device__ __forceinline__ void store(short (*Xs)[GKP], int t) const {
#pragma unroll
    for (int b = 0; b < NB; b++) {
      int rg, kg;
      if (!at(t + 256 * b, rg, kg)) continue;
#pragma unroll
      for (int r = 0; r < 4; r++)
        *(uint2 *)&Xs[4 * rg + r][4 * kg] =
            make_uint2(bf16_pair(v[b][0][r], v[b][1][r]), bf16_pair(v[b][2][r], v[b][3][r]));
    }
  }
};

template <int BT, bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float *__restrict__ A, int lda,
                                                   const float *__restrict__ B, int ldb, float *__restrict__ C,
                                                   int ldc, float alpha, float beta, int avec, int bvec) {
  constexpr int WT = BT / 2, MI = WT / 16;  // wave quadrant, MFMA tiles per side
  constexpr int GK = kstep(BT), GKP = GK + 8;
  __shared__ __attribute__((aligned(16))) short As[2][BT][GKP];  // [buf][m][k]
  __shared__ __attribute__((aligned(16))) short Bs[2][BT][GKP];  // [buf][n][k]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int m0 = blockIdx.y * BT, n0 = blockIdx.x * BT;
  const int wm = (wave >> 1) * WT, wn = (wave & 1) * WT;
  f32x4 acc[MI][MI];
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < MI; j++) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
  Slab<BT, !TA> sa;
  Slab<BT, TB> sb;
  sa.load(A, lda, M, K, m0, 0, avec, t);
  sb.load(B, ldb, N, K, n0, 0, bvec, t);
  sa.store(As[0], t);
  sb.store(Bs[0], t);
  __syncthreads();
  // operand fragments: row (m or n) = lane % 16, k = 8 (lane / 16) + i
  const int r16 = lane & 15, kb = (lane >> 4) * 8;
  const int nsteps = (K + GK - 1) / GK;
  for (int s = 0; s < nsteps; s++) {
    const int cur = s & 1;
    const bool more = s + 1 < nsteps;
    if (more) {
      sa.load(A, lda, M, K, m0, (s + 1) * GK, avec, t);
      sb.load(B, ldb, N, K, n0, (s + 1) * GK, bvec, t);
    }
#pragma unroll
    for (int kk = 0; kk < GK; kk += 32) {
      bf16x8v a[MI], b[MI];
#pragma unroll
      for (int i = 0; i < MI; i++) {
        a[i] = __builtin_bit_cast(bf16x8v, *(const s16x8 *)&As[cur][wm + 16 * i + r16][kk + kb]);
        b[i] = __builtin_bit_cast(bf16x8v, *(const s16x8 *)&Bs[cur][wn + 16 * i + r16][kk + kb]);
      }
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < MI; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      sa.store(As[cur ^ 1], t);
      sb.store(Bs[cur ^ 1], t);
    }
    __syncthreads();
  }
  // D layout: row = 4 (lane / 16) + q, column = lane % 16
  const int c16 = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < MI; j++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int gm = m0 + wm + 16 * i + rb + q, gn = n0 + wn + 16 * j + c16;
        if (gm < M && gn < N) {
          float *p = C + (int64_t)gm * ldc + gn;
          const float v = alpha * acc[i][j][q];
          *p = beta == 0.f ? v : fmaf(beta, *p, v);
        }
      }
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
// Phi(x) + x phi(x)
__device__ __forceinline__ float gelu_d(float x) {
  const float phi = 0.39894228040143268f * expf(-0.5f * x * x);
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * phi;
}
// phi(x) (2 - x^2)
__device__ __forceinline__ float gelu_dd(float x) {
  const float phi = 0.39894228040143268f * expf(-0.5f * x * x);
  return phi * (2.f - x * x);
}

// Z[m][j] += bias[j]; H = gelu(Z)  (row-major M x N)
__global__ void k_bias_gelu(int M, int N, float *__restrict__ Z, const float *__restrict__ bias, float *__restrict__ H) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const float z = Z[i] + bias[i % N];
  Z[i] = z;
  H[i] = gelu_f(z);
}

// elementwise helpers on M x N arrays; op selects the formula
//  0: out = gelu'(z) * v           1: out += gelu''(z) * u * v
//  2: out = gelu'(z) * w[col]      3: out += gelu''(z) * w[col] * v
//  4: out += gelu'(z) * v           5: out = gelu''(z) * u * v
//  6: out = gelu''(z) * w[col] * v
__global__ void k_ew(int op, int M, int N, const float *__restrict__ Z, const float *__restrict__ u,
                     const float *__restrict__ v, const float *__restrict__ w, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const float z = Z[i];
  switch (op) {
    case 0: out[i] = gelu_d(z) * v[i]; break;
    case 1: out[i] += gelu_dd(z) * u[i] * v[i]; break;
    case 2: out[i] = gelu_d(z) * w[i % N]; break;
    case 3: out[i] += gelu_dd(z) * w[i % N] * v[i]; break;
    case 5: out[i] = gelu_dd(z) * u[i] * v[i]; break;
    case 6: out[i] = gelu_dd(z) * w[i % N] * v[i]; break;
    default: out[i] += gelu_d(z) * v[i]; break;
  }
}

// y[m] = H[m] . w + b (N <= 1024): one block per row, fixed-order tree
__global__ void __launch_bounds__(256) k_rowdot(int M, int N, const float *__restrict__ H, const float *__restrict__ w,
                                               const float *__restrict__ b, float *__restrict__ y) {
  __shared__ float sh[256];
  const int m = blockIdx.x, t = threadIdx.x;
  float s = 0.f;
  for (int j = t; j < N; j += 256) s = fmaf(H[(int64_t)m * N + j], w[j], s);
  sh[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  if (t == 0) y[m] = sh[0] + (b ? b[0] : 0.f);
}

// out[j] (+)= scale * sum_m X[m][j] (column sums in a fixed order): a block
// covers 64 columns (one per lane, coalesced rows); its 16 waves take rows
// w, w + 16, ... into four running sums (independent loads in flight), and
// the waves' partial sums are added in wave order
constexpr int kColWaves = 16;
__global__ void __launch_bounds__(64 * kColWaves) k_colsum(int M, int N, const float *__restrict__ X, float scale,
                                                           int accumulate, float *__restrict__ out) {
  __shared__ float part[kColWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < N) {
    constexpr int S = kColWaves;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int m = w;
    for (; m + 3 * S < M; m += 4 * S) {
      s0 += X[(int64_t)m * N + j];
      s1 += X[(int64_t)(m + S) * N + j];
      s2 += X[(int64_t)(m + 2 * S) * N + j];
      s3 += X[(int64_t)(m + 3 * S) * N + j];
    }
    for (; m < M; m += S) s0 += X[(int64_t)m * N + j];
    s = (s0 + s1) + (s2 + s3);
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < N) {
    float r = 0.f;
    for (int v = 0; v < kColWaves; v++) r += part[v][lane];
    out[j] = accumulate ? out[j] + scale * r : scale * r;
  }
}

// out[m][j] = a[m] * w[j]  (outer product of a column vector and a row)
__global__ void k_outer(int M, int N, const float *__restrict__ a, const float *__restrict__ w, float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  out[i] = a[i / N] * w[i % N];
}

// r = scale * (g - G) over M x N
__global__ void k_axpby(int64_t n, float a, const float *x, float b, const float *y, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a * x[i] + (y ? b * y[i] : 0.f);
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * mhat / (sqrt(vhat) + eps)
__global__ void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static int blocks_for(int64_t n) { return (int)((n + 255) / 256); }

hipError_t mlp_gemm(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb, float *C,
                    int ldc, float alpha, float beta, hipStream_t st);
hipError_t mlp_bias_gelu(int M, int N, float *Z, const float *b, float *H, hipStream_t st);
hipError_t mlp_ew(int op, int M, int N, const float *Z, const float *u, const float *v, const float *w, float *out,
                  hipStream_t st);
hipError_t mlp_rowdot(int M, int N, const float *H, const float *w, const float *b, float *y, hipStream_t st);
hipError_t mlp_colsum(int M, int N, const float *X, float scale, int acc, float *out, hipStream_t st);
hipError_t mlp_outer(int M, int N, const float *a, const float *w, float *out, hipStream_t st);
hipError_t mlp_axpby(int64_t n, float a, const float *x, float b, const float *y, float *out, hipStream_t st);
hipError_t mlp_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st);

// ---------------------------------------------------------------- network

struct Mlp {
  int in, h1, h2, maxb;
  hipStream_t st;
  float *p = nullptr, *g = nullptr, *m1 = nullptr, *m2 = nullptr, *ws = nullptr;
  size_t np = 0;
  // parameter views
  float *W1, *b1, *W2, *b2, *w3, *b3;
  float *gW1, *gb1, *gW2, *gb2, *gw3, *gb3;
  // activations [maxb][*]
  float *Z1, *H1, *Z2, *H2, *A1, *A2, *U, *Gx, *R, *dA1, *dU, *dZ1, *dA2, *dZ2, *dH1, *T, *y, *dy;
};

}  // namespace vqc

struct vqc_mlp_s : vqc::Mlp {};

namespace vqc {

static hipError_t forward_impl(Mlp &m, int B, const float *x, bool want_dx) {
  hipStream_t st = m.st;
  hipError_t e;
  // Z1 = x W1^T + b1, H1 = gelu(Z1)
  if ((e = mlp_gemm(B, m.h1, m.in, x, m.in, 0, m.W1, m.in, 1, m.Z1, m.h1, 1.f, 0.f, st))) return e;
  if ((e = mlp_bias_gelu(B, m.h1, m.Z1, m.b1, m.H1, st))) return e;
  if ((e = mlp_gemm(B, m.h2, m.h1, m.H1, m.h1, 0, m.W2, m.h1, 1, m.Z2, m.h2, 1.f, 0.f, st))) return e;
  if ((e = mlp_bias_gelu(B, m.h2, m.Z2, m.b2, m.H2, st))) return e;
  if ((e = mlp_rowdot(B, m.h2, m.H2, m.w3, m.b3, m.y, st))) return e;
  if (!want_dx) return hipSuccess;
  // A2 = gelu'(Z2) w3, U = A2 W2, A1 = gelu'(Z1) U, Gx = A1 W1
  if ((e = mlp_ew(2, B, m.h2, m.Z2, nullptr, nullptr, m.w3, m.A2, st))) return e;
  if ((e = mlp_gemm(B, m.h1, m.h2, m.A2, m.h2, 0, m.W2, m.h1, 0, m.U, m.h1, 1.f, 0.f, st))) return e;
  if ((e = mlp_ew(0, B, m.h1, m.Z1, nullptr, m.U, nullptr, m.A1, st))) return e;
  return mlp_gemm(B, m.in, m.h1, m.A1, m.h1, 0, m.W1, m.in, 0, m.Gx, m.in, 1.f, 0.f, st);
}

static hipError_t backward_impl(Mlp &m, int B, const float *x, const float *E, const float *G, float lambda) {
  hipStream_t st = m.st;
  hipError_t e;
  const bool sob = G && lambda != 0.f;
  if ((e = forward_impl(m, B, x, sob))) return e;
  float beta = 0.f;  // first write of each weight gradient overwrites
  if (sob) {
    // R = 2 lambda / (B n_in) (Gx - G)
    const float s = 2.f * lambda / ((float)B * m.in);
    if ((e = mlp_axpby((int64_t)B * m.in, s, m.Gx, -s, G, m.R, st))) return e;
    // Gx = A1 W1: dW1 = A1^T R, dA1 = R W1^T
    if ((e = mlp_gemm(m.h1, m.in, B, m.A1, m.h1, 1, m.R, m.in, 0, m.gW1, m.in, 1.f, 0.f, st))) return e;
    if ((e = mlp_gemm(B, m.h1, m.in, m.R, m.in, 0, m.W1, m.in, 1, m.dA1, m.h1, 1.f, 0.f, st))) return e;
    // A1 = gelu'(Z1) U: dU = gelu'(Z1) dA1, dZ1 = gelu''(Z1) U dA1
    if ((e = mlp_ew(0, B, m.h1, m.Z1, nullptr, m.dA1, nullptr, m.dU, st))) return e;
    if ((e = mlp_ew(5, B, m.h1, m.Z1, m.U, m.dA1, nullptr, m.dZ1, st))) return e;
    // U = A2 W2: dW2 = A2^T dU, dA2 = dU W2^T
    if ((e = mlp_gemm(m.h2, m.h1, B, m.A2, m.h2, 1, m.dU, m.h1, 0, m.gW2, m.h1, 1.f, 0.f, st))) return e;
    if ((e = mlp_gemm(B, m.h2, m.h1, m.dU, m.h1, 0, m.W2, m.h1, 1, m.dA2, m.h2, 1.f, 0.f, st))) return e;
    // A2 = gelu'(Z2) w3: dw3 = sum_b gelu'(Z2) dA2, dZ2 = gelu''(Z2) w3 dA2
    if ((e = mlp_ew(0, B, m.h2, m.Z2, nullptr, m.dA2, nullptr, m.T, st))) return e;
    if ((e = mlp_colsum(B, m.h2, m.T, 1.f, 0, m.gw3, st))) return e;
    if ((e = mlp_ew(6, B, m.h2, m.Z2, nullptr, m.dA2, m.w3, m.dZ2, st))) return e;
    beta = 1.f;
  }
  // energy term: dy = 2/B (y - E)
  if ((e = mlp_axpby(B, 2.f / B, m.y, -2.f / B, E, m.dy, st))) return e;
  // y = H2 w3 + b3: dw3 += dy^T H2, db3 = sum dy, dH2 = dy w3^T
  if ((e = mlp_gemm(1, m.h2, B, m.dy, B, 0, m.H2, m.h2, 0, m.gw3, m.h2, 1.f, beta, st))) return e;
  if ((e = mlp_colsum(B, 1, m.dy, 1.f, 0, m.gb3, st))) return e;
  if ((e = mlp_outer(B, m.h2, m.dy, m.w3, m.T, st))) return e;
  // dZ2 (+)= gelu'(Z2) dH2
  if (sob) {
    if ((e = mlp_ew(4, B, m.h2, m.Z2, nullptr, m.T, nullptr, m.dZ2, st))) return e;
  } else {
    if ((e = mlp_ew(0, B, m.h2, m.Z2, nullptr, m.T, nullptr, m.dZ2, st))) return e;
  }
  // Z2 = H1 W2^T + b2: db2 = sum dZ2, dW2 (+)= dZ2^T H1, dH1 = dZ2 W2
  if ((e = mlp_colsum(B, m.h2, m.dZ2, 1.f, 0, m.gb2, st))) return e;
  if ((e = mlp_gemm(m.h2, m.h1, B, m.dZ2, m.h2, 1, m.H1, m.h1, 0, m.gW2, m.h1, 1.f, beta, st))) return e;
  if ((e = mlp_gemm(B, m.h1, m.h2, m.dZ2, m.h2, 0, m.W2, m.h1, 0, m.dH1, m.h1, 1.f, 0.f, st))) return e;
  if (sob) {
    if ((e = mlp_ew(4, B, m.h1, m.Z1, nullptr, m.dH1, nullptr, m.dZ1, st))) return e;
  } else {
    if ((e = mlp_ew(0, B, m.h1, m.Z1, nullptr, m.dH1, nullptr, m.dZ1, st))) return e;
  }
  // Z1 = x W1^T + b1: db1 = sum dZ1, dW1 (+)= dZ1^T x
  if ((e = mlp_colsum(B, m.h1, m.dZ1, 1.f, 0, m.gb1, st))) return e;
  return mlp_gemm(m.h1, m.in, B, m.dZ1, m.h1, 1, x, m.in, 0, m.gW1, m.in, 1.f, beta, st);
}

}  // namespace vqc

using namespace vqc;

static vqc_status hst(hipError_t e) {
  if (e == hipSuccess) return VQC_OK;
  return e == hipErrorOutOfMemory ? VQC_ERR_OOM : VQC_ERR_HIP;
}

extern "C" {

vqc_status vqc_gemm_bf16(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb,
                         float *C, int ldc, float alpha, float beta, void *stream) {
  if (M < 0 || N < 0 || K < 0 || !A || !B || !C || lda < 1 || ldb < 1 || ldc < 1) return VQC_ERR_ARG;
  if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) return VQC_ERR_ARG;
  if (lda < (ta ? M : K) || ldb < (tb ? K : N) || ldc < N) return VQC_ERR_ARG;
  return hst(mlp_gemm(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, (hipStream_t)stream));
}

vqc_status vqc_mlp_create(vqc_mlp *out, int n_in, int h1, int h2, int max_batch, void *stream) {
  if (!out || n_in < 1 || h1 < 1 || h2 < 1 || h2 > 1 << 16 || max_batch < 1) return VQC_ERR_ARG;
  vqc_mlp m = new (std::nothrow) vqc_mlp_s();
  if (!m) return VQC_ERR_OOM;
  m->in = n_in;
  m->h1 = h1;
  m->h2 = h2;
  m->maxb = max_batch;
  m->st = (hipStream_t)stream;
  m->np = (size_t)h1 * n_in + h1 + (size_t)h2 * h1 + h2 + h2 + 1;
  const size_t B = max_batch, hm = (size_t)(h1 > h2 ? h1 : h2), wide = hm > (size_t)n_in ? hm : n_in;
  const size_t nws = 18 * B * wide + 2 * B;
  hipError_t e = hipMalloc(&m->p, 4 * m->np * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->ws, nws * sizeof(float));
  if (e != hipSuccess) {
    if (m->p) (void)hipFree(m->p);
    delete m;
    return hst(e);
  }
  m->g = m->p + m->np;
  m->m1 = m->g + m->np;
  m->m2 = m->m1 + m->np;
  float *q = m->p;
  m->W1 = q; q += (size_t)h1 * n_in;
  m->b1 = q; q += h1;
  m->W2 = q; q += (size_t)h2 * h1;
  m->b2 = q; q += h2;
  m->w3 = q; q += h2;
  m->b3 = q;
  q = m->g;
  m->gW1 = q; q += (size_t)h1 * n_in;
  m->gb1 = q; q += h1;
  m->gW2 = q; q += (size_t)h2 * h1;
  m->gb2 = q; q += h2;
  m->gw3 = q; q += h2;
  m->gb3 = q;
  float *w = m->ws;
  float **acts[] = {&m->Z1, &m->H1, &m->Z2, &m->H2, &m->A1, &m->A2, &m->U, &m->Gx, &m->R,
                    &m->dA1, &m->dU, &m->dZ1, &m->dA2, &m->dZ2, &m->dH1, &m->T};
  for (float **a : acts) { *a = w; w += B * wide; }
  m->y = w; w += B;
  m->dy = w;
  e = hipMemsetAsync(m->m1, 0, 2 * m->np * sizeof(float), m->st);
  if (e == hipSuccess) e = hipStreamSynchronize(m->st);
  if (e != hipSuccess) {
    vqc_mlp_destroy(m);
    return hst(e);
  }
  *out = m;
  return VQC_OK;
}

vqc_status vqc_mlp_destroy(vqc_mlp m) {
  if (!m) return VQC_OK;
  if (m->p) (void)hipFree(m->p);
  if (m->ws) (void)hipFree(m->ws);
  delete m;
  return VQC_OK;
}

vqc_status vqc_mlp_buffers(vqc_mlp m, float **params, float **grads, size_t *count) {
  if (!m) return VQC_ERR_ARG;
  if (params) *params = m->p;
  if (grads) *grads = m->g;
  if (count) *count = m->np;
  return VQC_OK;
}

vqc_status vqc_mlp_forward(vqc_mlp m, int batch, const float *x, float *y, float *dydx) {
  if (!m || !x || !y || batch < 1 || batch > m->maxb) return VQC_ERR_ARG;
  hipError_t e = forward_impl(*m, batch, x, dydx != nullptr);
  if (e == hipSuccess) e = hipMemcpyAsync(y, m->y, batch * sizeof(float), hipMemcpyDeviceToDevice, m->st);
  if (e == hipSuccess && dydx)
    e = hipMemcpyAsync(dydx, m->Gx, (size_t)batch * m->in * sizeof(float), hipMemcpyDeviceToDevice, m->st);
  return hst(e);
}

vqc_status vqc_mlp_backward(vqc_mlp m, int batch, const float *x, const float *E, const float *G, float lambda,
                            float *y, float *dydx) {
  if (!m || !x || !E || batch < 1 || batch > m->maxb) return VQC_ERR_ARG;
  hipError_t e = backward_impl(*m, batch, x, E, G, lambda);
  if (e == hipSuccess && y) e = hipMemcpyAsync(y, m->y, batch * sizeof(float), hipMemcpyDeviceToDevice, m->st);
  if (e == hipSuccess && dydx && G && lambda != 0.f)
    e = hipMemcpyAsync(dydx, m->Gx, (size_t)batch * m->in * sizeof(float), hipMemcpyDeviceToDevice, m->st);
  return hst(e);
}

vqc_status vqc_mlp_adam(vqc_mlp m, float lr, float b1, float b2, float eps, int step) {
  if (!m || step < 1) return VQC_ERR_ARG;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  return hst(mlp_adam((int64_t)m->np, m->p, m->g, m->m1, m->m2, lr, b1, b2, eps, c1, c2, m->st));
}

vqc_status vqc_mlp_descend_inputs(vqc_mlp m, int batch, float *x, float lr, int steps) {
  if (!m || !x || batch < 1 || batch > m->maxb || steps < 0) return VQC_ERR_ARG;
  for (int s = 0; s < steps; s++) {
    hipError_t e = forward_impl(*m, batch, x, true);
    if (e == hipSuccess) e = mlp_axpby((int64_t)batch * m->in, 1.f, x, -lr, m->Gx, x, m->st);
    if (e != hipSuccess) return hst(e);
  }
  return VQC_OK;
}

}  // extern "C"

namespace vqc {

template <int BT>
static void launch_gemm_t(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb,
                          float *C, int ldc, float alpha, float beta, int avec, int bvec, hipStream_t st) {
  dim3 grid((N + BT - 1) / BT, (M + BT - 1) / BT);
#define VQC_GEMM_LAUNCH(TA, TB)                                                                                    \
  hipLaunchKernelGGL((k_gemm_bf16<BT, TA, TB>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, alpha, beta, \
                     avec, bvec)
  if (!ta && !tb) VQC_GEMM_LAUNCH(false, false);
  else if (ta && !tb) VQC_GEMM_LAUNCH(true, false);
  else if (!ta && tb) VQC_GEMM_LAUNCH(false, true);
  else VQC_GEMM_LAUNCH(true, true);
#undef VQC_GEMM_LAUNCH
}

hipError_t mlp_gemm(int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb, float *C,
                    int ldc, float alpha, float beta, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // float4 loads need a 16-byte aligned base and a leading dimension that keeps every row aligned
  const int avec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  const int bvec = ((uintptr_t)B % 16 == 0) && (ldb % 4 == 0);
  // the largest tile whose grid still gives every compute unit a block
  auto blocks = [&](int bt) { return (int64_t)((M + bt - 1) / bt) * ((N + bt - 1) / bt); };
  if (blocks(128) >= 256)
    launch_gemm_t<128>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, avec, bvec, st);
  else if (blocks(64) >= 128)
    launch_gemm_t<64>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, avec, bvec, st);
  else
    launch_gemm_t<32>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, avec, bvec, st);
  return hipGetLastError();
}
hipError_t mlp_bias_gelu(int M, int N, float *Z, const float *b, float *H, hipStream_t st) {
  hipLaunchKernelGGL(k_bias_gelu, dim3(blocks_for((int64_t)M * N)), dim3(256), 0, st, M, N, Z, b, H);
  return hipGetLastError();
}
hipError_t mlp_ew(int op, int M, int N, const float *Z, const float *u, const float *v, const float *w, float *out,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_ew, dim3(blocks_for((int64_t)M * N)), dim3(256), 0, st, op, M, N, Z, u, v, w, out);
  return hipGetLastError();
}
hipError_t mlp_rowdot(int M, int N, const float *H, const float *w, const float *b, float *y, hipStream_t st) {
  hipLaunchKernelGGL(k_rowdot, dim3(M), dim3(256), 0, st, M, N, H, w, b, y);
  return hipGetLastError();
}
hipError_t mlp_colsum(int M, int N, const float *X, float scale, int acc, float *out, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(64 * kColWaves), 0, st, M, N, X, scale, acc, out);
  return hipGetLastError();
}
hipError_t mlp_outer(int M, int N, const float *a, const float *w, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_outer, dim3(blocks_for((int64_t)M * N)), dim3(256), 0, st, M, N, a, w, out);
  return hipGetLastError();
}
hipError_t mlp_axpby(int64_t n, float a, const float *x, float b, const float *y, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(256), 0, st, n, a, x, b, y, out);
  return hipGetLastError();
}
hipError_t mlp_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace vqc

// Dense products of the DINO training step (paper Sec. 3.4,
// eq. (reduced_basis_derivative_equivalence); Sec. 4.2.1): forward layers,
// forward-mode Jacobian tangents, and the hand-written reverse pass, all
// C = alpha op(A) op(B) + beta C on row-major FP32 arrays.
//
// Operands are rounded to BF16 (the training precision of the workload: BF16
// weights and activations, FP32 accumulation, FP32 master weights) or kept
// in FP32, and multiplied on the matrix cores:
//   BF16: v_mfma_f32_16x16x32_bf16, one 16 x 32 x 16 step per instruction;
//   FP32: v_mfma_f32_16x16x4_f32, eight instructions per 32-deep k step.
// Lane l of a 16 x 16 MFMA tile supplies row l % 16 of A and column l % 16 of
// B at depth offsets 8 (l / 16) .. +8 (BF16) or l / 16 (FP32), and receives
// rows 4 (l / 16) .. +4 of column l % 16 of the product.
//
// A 256-thread workgroup (4 waves, 2 x 2) owns a 64 x 64 output tile; each
// wave a 32 x 32 quarter (2 x 2 MFMA tiles).  Per 32-deep step both operand
// tiles are staged in LDS with k contiguous per row (BF16 rows padded to 40
// values, FP32 rows to 36, so the fragment reads of 16 rows fall into
// distinct banks); global loads are coalesced along whichever index is
// contiguous in memory, and the next step's values are loaded into registers
// while the current step multiplies.  Products with few output tiles and a
// long k (the weight gradients, k = batch x d_Z) are split along k into
// partial products that a second kernel sums in a fixed order, so results
// are bitwise reproducible.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "runtime.h"

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int GT_M = 64, GT_N = 64, GT_K = 32;

// Eight values of one operand tile per thread.  KC: the operand's k index is
// contiguous in memory (X[r * ld + k]); otherwise its row index is
// (X[k * ld + r]).  Out-of-range entries are zero.
template <bool KC>
__device__ __forceinline__ void gload(const float* __restrict__ X, int64_t ld, int R, int K, int r0, int k0,
                                      float (&v)[8], int tid) {
  if constexpr (KC) {
    const int kk = tid & 31, rr = tid >> 5;
    const int k = k0 + kk;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int r = r0 + rr + 8 * i;
      v[i] = (r < R && k < K) ? X[(int64_t)r * ld + k] : 0.0f;
    }
  } else {
    const int rr = tid & 63, kk = tid >> 6;
    const int r = r0 + rr;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + kk + 4 * i;
      v[i] = (r < R && k < K) ? X[(int64_t)k * ld + r] : 0.0f;
    }
  }
}

template <bool KC, typename T, int LD>
__device__ __forceinline__ void gstore(T* __restrict__ S, const float (&v)[8], int tid) {
  if constexpr (KC) {
    const int kk = tid & 31, rr = tid >> 5;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[(rr + 8 * i) * LD + kk] = (T)v[i];
  } else {
    const int rr = tid & 63, kk = tid >> 6;
#pragma unroll
    for (int i = 0; i < 8; ++i) S[rr * LD + kk + 4 * i] = (T)v[i];
  }
}

}  // namespace

// C (or, with part != nullptr, the partial product of k slice blockIdx.z into
// part[z][M][N]) for the 64 x 64 tile (blockIdx.y, blockIdx.x).
template <bool BF, bool TA, bool TB>
__global__ __launch_bounds__(256) void saa_k_gemm(int M, int N, int K, int kchunk, float alpha,
                                                  const float* __restrict__ A, int lda, const float* __restrict__ B,
                                                  int ldb, float beta, float* __restrict__ C, int ldc,
                                                  float* __restrict__ part) {
  typedef typename std::conditional<BF, __bf16, float>::type T;
  constexpr int LD = BF ? 40 : 36;
  __shared__ __attribute__((aligned(16))) T As[GT_M * LD];
  __shared__ __attribute__((aligned(16))) T Bs[GT_N * LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * GT_M, n0 = blockIdx.x * GT_N;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  // op(A)[m][k] is k-contiguous unless A is transposed; op(B)[k][n] is
  // k-contiguous only when B is transposed
  constexpr bool AKC = !TA, BKC = TB;
  f32x4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4_t){0.0f, 0.0f, 0.0f, 0.0f};
  float ra[8], rb[8];
  if (kb < ke) {
    gload<AKC>(A, lda, M, K, m0, kb, ra, tid);
    gload<BKC>(B, ldb, N, K, n0, kb, rb, tid);
  }
  const int fr = lane & 15, fg = lane >> 4;
  for (int k0 = kb; k0 < ke; k0 += GT_K) {
    __syncthreads();
    gstore<AKC, T, LD>(As, ra, tid);
    gstore<BKC, T, LD>(Bs, rb, tid);
    __syncthreads();
    if (k0 + GT_K < ke) {
      gload<AKC>(A, lda, M, K, m0, k0 + GT_K, ra, tid);
      gload<BKC>(B, ldb, N, K, n0, k0 + GT_K, rb, tid);
    }
    if constexpr (BF) {
      bf16x8_t fa[2], fb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        fa[t] = *(const bf16x8_t*)&As[(wm * 32 + t * 16 + fr) * LD + 8 * fg];
        fb[t] = *(const bf16x8_t*)&Bs[(wn * 32 + t * 16 + fr) * LD + 8 * fg];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    } else {
#pragma unroll
      for (int s = 0; s < GT_K / 4; ++s) {
        float fa[2], fb[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          fa[t] = As[(wm * 32 + t * 16 + fr) * LD + 4 * s + fg];
          fb[t] = Bs[(wn * 32 + t * 16 + fr) * LD + 4 * s + fg];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  float* P = part ? part + (int64_t)blockIdx.z * M * N : nullptr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int n = n0 + wn * 32 + b * 16 + fr;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = m0 + wm * 32 + a * 16 + 4 * fg + i;
        if (m >= M || n >= N) continue;
        const float v = acc[a][b][i];
        if (P) {
          P[(int64_t)m * N + n] = v;
        } else {
          float* c = C + (int64_t)m * ldc + n;
          *c = beta != 0.0f ? alpha * v + beta * *c : alpha * v;
        }
      }
    }
}

// C = alpha sum_z part[z] + beta C, the slices summed in increasing z.
__global__ void saa_k_gemm_reduce(int M, int N, int splits, float alpha, const float* __restrict__ part, float beta,
                                  float* __restrict__ C, int ldc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = (int64_t)M * N;
  if (t >= MN) return;
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * MN + t];
  const int m = (int)(t / N), n = (int)(t % N);
  float* c = C + (int64_t)m * ldc + n;
  *c = beta != 0.0f ? alpha * s + beta * *c : alpha * s;
}

namespace saa_launch {

// Row-major C[M x N] = alpha op(A) op(B) + beta C with op(A) = A (M x K,
// leading dimension lda) or A^T (A stored K x M), op(B) = B (K x N) or B^T
// (B stored N x K).  bf16: operands rounded to BF16, else FP32; FP32
// accumulation either way.  ws (ws_floats floats, may be null) holds the
// partial products of a k split.  With beta = 0, C is not read.
int gemm_mfma(bool bf16, bool ta, bool tb, int M, int N, int K, float alpha, const float* A, int lda, const float* B,
              int ldb, float beta, float* C, int ldc, float* ws, int64_t ws_floats, hipStream_t st) {
  if (M < 0 || N < 0 || K < 0) return SAA_E_INVALID;
  if (M == 0 || N == 0) return SAA_OK;
  const int tm = (M + GT_M - 1) / GT_M, tn = (N + GT_N - 1) / GT_N;
  const int64_t tiles = (int64_t)tm * tn;
  int splits = 1;
  if (ws && tiles < 128 && K >= 512) {
    splits = (int)std::min<int64_t>((256 + tiles - 1) / tiles, K / 256);
    splits = (int)std::min<int64_t>(splits, ws_floats / ((int64_t)M * N));
    splits = std::max(splits, 1);
  }
  int kchunk = (K + splits - 1) / splits;
  kchunk = std::max(GT_K, (kchunk + GT_K - 1) / GT_K * GT_K);
  splits = std::max(1, (K + kchunk - 1) / kchunk);
  float* part = splits > 1 ? ws : nullptr;
  const dim3 grid(tn, tm, splits);
#define SAA_GEMM_LAUNCH(BFv, TAv, TBv) \
  saa_k_gemm<BFv, TAv, TBv><<<grid, 256, 0, st>>>(M, N, K, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, part)
  if (bf16) {
    if (!ta && !tb) SAA_GEMM_LAUNCH(true, false, false);
    else if (!ta && tb) SAA_GEMM_LAUNCH(true, false, true);
    else if (ta && !tb) SAA_GEMM_LAUNCH(true, true, false);
    else SAA_GEMM_LAUNCH(true, true, true);
  } else {
    if (!ta && !tb) SAA_GEMM_LAUNCH(false, false, false);
    else if (!ta && tb) SAA_GEMM_LAUNCH(false, false, true);
    else if (ta && !tb) SAA_GEMM_LAUNCH(false, true, false);
    else SAA_GEMM_LAUNCH(false, true, true);
  }
#undef SAA_GEMM_LAUNCH
  if (part) {
    const int64_t MN = (int64_t)M * N;
    saa_k_gemm_reduce<<<(unsigned)((MN + 255) / 256), 256, 0, st>>>(M, N, splits, alpha, part, beta, C, ldc);
  }
  return saa_rt::check_hip(hipGetLastError());
}

}  // namespace saa_launch

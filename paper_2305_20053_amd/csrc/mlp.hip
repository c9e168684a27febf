// MR-DINO surrogate evaluation (paper Sec. 3.3, eq. (rbnet); Sec. 3.1,
// eq. (neural_operator_risk) / (neural_operator_gradient)):
//
//   x = [xi_hat (r_m leading KL coordinates); z]
//   a_L = W_L h_{L-1} + b_L, h_L = GELU(a_L), L = 0..depth-1;  phi = W_depth h + b
//   q = |phi + c|^2 + c0                 (reduced quadratic QoI, Sec. 3.3)
//   dq/dz by reverse mode: delta = 2 (phi + c), back through the layers with
//   GELU'(a_L), and finally the control columns of W_0.
//
// MFMA kernel (v_mfma_f32_16x16x32_bf16, or v_mfma_scale_f32_16x16x128_f8f6f4
// on E4M3 operands; FP32 accumulation).
// Products are formed transposed, C = W_L * H^T: output features run along
// the MFMA M dimension and samples along N, so one lane holds, for its sample,
// 4 consecutive features of every 16-feature tile.  That accumulator layout is
// the B-operand layout of the next layer up to a fixed permutation inside
// every 32-feature block (slot 8g + t holds feature 4g + t for t < 4 and
// 16 + 4g + t - 4 for t >= 4); the permutation is folded into the stored
// weight copies, so a lane's outputs are published to the next product
// without any shuffle.  A workgroup carries 64 samples and splits every
// product's output features over its waves (see the kernel).  GELU'(a_L) of
// every layer is kept in LDS as fp16 for the reverse pass.
//
// The weights (A operands) are stored once per format, every 16 x 32 fragment
// contiguous (64 lanes x 16 B for BF16), in the order
// wp[0..depth], wt[depth..1], w0z; a wave reads its fragments straight from
// L2, where the whole set (1.1 MB in BF16) stays resident.
#include <hip/hip_fp16.h>

#include <string>
#include <type_traits>

#include "common.h"
#include "mlp.h"
#include "tune.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef long i64x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int kperm(int k) {
  const int b = k & ~31, kk = k & 31, g = kk >> 3, t = kk & 7;
  return b + (t < 4 ? 4 * g + t : 16 + 4 * g + (t - 4));
}

// GELU and its derivative of two pre-activations for the MFMA kernels,
// branch-free, in packed FP16 (v_pk_fma_f16 and friends; exp2 and rcp per
// half): Phi(a) = (1 + erf(a / sqrt 2)) / 2 with erf from Abramowitz & Stegun
// (1964), formula 7.1.26 (absolute error <= 1.5e-7); the factor exp(-a^2 / 2)
// is shared with GELU'(a) = Phi(a) + a phi(a).  The kernels round h to BF16
// / FP8 for the next product and keep GELU' as fp16, so FP16 arithmetic
// (relative rounding 4.9e-4) stays below those roundings.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void gelu_pair2(float a0, float a1, float& h0, float& h1, _Float16& d0, _Float16& d1) {
  const h2v a = {(_Float16)a0, (_Float16)a1};
  const h2v x = __builtin_elementwise_abs(a) * (h2v)(_Float16)0.70710678f;
  const h2v den = __builtin_elementwise_fma((h2v)(_Float16)0.3275911f, x, (h2v)(_Float16)1.0f);
  const h2v t = {(_Float16)__builtin_amdgcn_rcph(den.x), (_Float16)__builtin_amdgcn_rcph(den.y)};
  h2v p = __builtin_elementwise_fma(t, (h2v)(_Float16)1.061405429f, (h2v)(_Float16)-1.453152027f);
  p = __builtin_elementwise_fma(p, t, (h2v)(_Float16)1.421413741f);
  p = __builtin_elementwise_fma(p, t, (h2v)(_Float16)-0.284496736f);
  p = __builtin_elementwise_fma(p, t, (h2v)(_Float16)0.254829592f);
  p = p * t;
  const h2v e = __builtin_elementwise_exp2((x * x) * (h2v)(_Float16)-1.44269504f);   // exp(-x^2)
  const h2v erfx = __builtin_elementwise_fma(-p, e, (h2v)(_Float16)1.0f);
  const h2v phi = __builtin_elementwise_fma(__builtin_elementwise_copysign(erfx, a), (h2v)(_Float16)0.5f,
                                            (h2v)(_Float16)0.5f);   // Phi(a)
  const h2v h = a * phi;
  const h2v dh = __builtin_elementwise_fma(a * (h2v)(_Float16)0.39894228f, e, phi);
  h0 = (float)h.x;
  h1 = (float)h.y;
  d0 = dh.x;
  d1 = dh.y;
}

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float dgelu_f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

// Operand formats of the fused kernel.  Outputs are exchanged through LDS
// as 16 x 32 blocks (lane 16 g + c: row / column c, k = 8 g .. 8 g + 8):
//  OpBF16: BF16 values, 1 KB per block, one v_mfma_f32_16x16x32_bf16 per
//          block;
//  OpFP8:  FP8 (E4M3) values, 512 B per block; one
//          v_mfma_scale_f32_16x16x128_f8f6f4 takes four consecutive blocks
//          (a lane's 32 bytes are its 8 bytes of each, in order; the weight
//          copy stores them contiguously, 2 KB per 16 x 128 fragment).
//          Weights carry a power-of-two scale per operand, activations one
//          per sample (from the largest magnitude of the sample's features);
//          the MFMA undoes both through its E8M0 operand scales, so only the
//          3-bit mantissa rounding remains.
struct OpBF16 {
  typedef bf16x8 vec;
  static constexpr int FB = 1024;
  static constexpr bool scaled = false;
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static vec pack(const float (&v)[8], float) {
    vec r;
#pragma unroll
    for (int t = 0; t < 8; ++t) r[t] = (__bf16)v[t];
    return r;
  }
};
struct OpFP8 {
  typedef long vec;
  static constexpr int FB = 512;
  static constexpr bool scaled = true;
  // sa, sb: E8M0 scale (2^(s - 127)) of the lane's A row / B column
  __device__ static f32x4 mma4(i32x8 a, i32x8 b, f32x4 c, int sa, int sb) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
  }
  __device__ static vec pack(const float (&v)[8], float s) {
    int lo = 0, hi = 0;
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0] * s, v[1] * s, lo, false);
    lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2] * s, v[3] * s, lo, true);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4] * s, v[5] * s, hi, false);
    hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6] * s, v[7] * s, hi, true);
    return (long)(unsigned)lo | ((long)hi << 32);
  }
};

// Exponent e of the power of two s = 2^e with m s in [top / 2, top) (0 for
// m = 0), clamped to [-60, 60]: the FP8 operand scale of values of largest
// magnitude m (E4M3 holds magnitudes up to 448).
__device__ __forceinline__ int pow2_exp(float m, float top) {
  if (!(m > 0.0f) || !(m < INFINITY)) return 0;
  int e;
  (void)frexpf(top / m, &e);
  return e - 1 < -60 ? -60 : (e - 1 > 60 ? 60 : e - 1);
}
__device__ __forceinline__ float pow2_scale(float m, float top) { return ldexpf(1.0f, pow2_exp(m, top)); }
// The same for top = 256 without a division: m = f 2^em with f in [0.5, 1)
// gives m 2^(8 - em) in [128, 256).
__device__ __forceinline__ int pow2_exp256(float m) {
  if (!(m > 0.0f) || !(m < INFINITY)) return 0;
  int em;
  (void)frexpf(m, &em);
  const int e = 8 - em;
  return e < -60 ? -60 : (e > 60 ? 60 : e);
}

}  // namespace

// ---------------------------------------------------------------------------
// Weight packing (after every change of the FP32 master parameters)
// ---------------------------------------------------------------------------

// Position t of a stored rows x cols operand (fragment (ks, mt) at
// ks * rows/16 + mt, 64 lanes x 8 values each) -> logical (row m, column k).
__device__ __forceinline__ void frag_pos(int64_t t, int rows, int& m, int& k) {
  const int e = (int)(t & 7);
  const int ln = (int)((t >> 3) & 63);
  const int64_t f = t >> 9;                // fragment index ks * (rows/16) + mt
  const int nmt = rows >> 4;
  const int ks = (int)(f / nmt), mt = (int)(f % nmt);
  m = 16 * mt + (ln & 15);
  k = 32 * ks + 8 * (ln >> 4) + e;
}

// Forward BF16 operand (fragment order): logical [m][k] = W[m][kperm(k)] (or
// natural order when `natural`), zero outside the source.  W is src_rows x
// src_ld.  rows % 16 == 0, cols % 32 == 0.
__global__ void saa_k_pack_fwd(__bf16* dst, const float* src, int rows, int cols, int src_rows, int src_cols,
                               int src_ld, int natural) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  int m, k;
  frag_pos(t, rows, m, k);
  const int ks = natural ? k : kperm(k);
  float v = 0.0f;
  if (m < src_rows && ks < src_cols) v = src[(int64_t)m * src_ld + ks];
  dst[t] = (__bf16)v;
}

// Backward BF16 operand (fragment order): logical [m][k] = W[kperm(k)][col0 + m],
// zero outside.
__global__ void saa_k_pack_bwd(__bf16* dst, const float* src, int rows, int cols, int src_rows, int src_cols,
                               int src_ld, int col0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  int m, k;
  frag_pos(t, rows, m, k);
  const int o = kperm(k);
  float v = 0.0f;
  if (o < src_rows && m < src_cols) v = src[(int64_t)o * src_ld + col0 + m];
  dst[t] = (__bf16)v;
}

// FP32 transpose: dst[k][m] = W[m][k] (W rows x cols).
__global__ void saa_k_transpose(float* dst, const float* src, int rows, int cols, int src_ld) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * cols) return;
  const int k = (int)(t / rows), m = (int)(t % rows);
  dst[t] = src[(int64_t)m * src_ld + k];
}

// Zero-padded copy of a vector.
__global__ void saa_k_pad(float* dst, const float* src, int n_src, int n_dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_dst) dst[t] = t < n_src ? src[t] : 0.0f;
}

// BF16 surrogate input of every installed sample: X[s][k] = xi_s[order[k]] for
// k < r_m, 0 up to kin (the leading KL coordinates, Sec. 3.3).  The samples
// are fixed, so this runs once per sample set.
__global__ void saa_k_encode(const double* xi, int nkl, const int* order, int r_m, int kin, int64_t N, __bf16* X) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * kin) return;
  const int64_t s = t / kin;
  const int k = (int)(t - s * kin);
  X[t] = (__bf16)(k < r_m ? (float)xi[s * nkl + order[k]] : 0.0f);
}

// dst[i] = a[i] + b[i] for i < n, 0 for n <= i < w.
__global__ void saa_k_add_pad(float* dst, const float* a, const float* b, int n, int w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < w) dst[i] = i < n ? a[i] + b[i] : 0.0f;
}

// b0eff[f] = b_0[f] + sum_k W_0[f][r_m + k] z_k  (the control enters only
// through the first layer and is shared by all samples).  W0zT is the packed
// transposed copy of those columns (d_z x width), so consecutive threads
// read consecutive features.
// z may live in pinned host memory (a replayed graph): the workgroup reads it
// once into LDS.
__global__ void __launch_bounds__(64) saa_k_b0eff(float* b0eff, const float* W0zT, const float* b0, const double* z,
                                                 int width, int d_z) {
  __shared__ float zs[64];
  if (threadIdx.x < d_z) zs[threadIdx.x] = (float)z[threadIdx.x];
  __syncthreads();
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= width) return;
  float acc = b0[f];
#pragma unroll 8
  for (int k = 0; k < d_z; ++k) acc += W0zT[(int64_t)k * width + f] * zs[k];
  b0eff[f] = acc;
}

// ---------------------------------------------------------------------------
// Fused MFMA kernel (forward, reduced QoI, reverse pass, dq/dz), feature split.
// A workgroup of WAVES waves carries 64 samples (4 blocks of 16); wave w
// computes output tiles MW w .. MW w + MW - 1 of every product for all 64
// samples, so each A fragment it loads (straight from L2, two k-steps ahead)
// feeds 4 MFMAs.  A wave's outputs are, lane by lane, whole B fragments of
// k-steps KW w .. of the next product (the k-permutation of the stored
// weights); they are exchanged through LDS (two barriers per layer).
// GELU'(a) stays with the wave that computed a, which is also the wave that
// needs it in the reverse pass.  Two waves per SIMD let one wave's GELU
// epilogue overlap the other's MFMAs.
// FP8: the activations of a sample share one power-of-two scale; each wave
// posts its per-sample maximum in LDS before the publishing barrier.  A
// product takes four 16 x 32 blocks per MFMA (16 x 16 x 128), the A operand
// from the 2 KB fragments of the FP8 stream, the B operand gathered from the
// four blocks in LDS; the scales travel as the MFMA's E8M0 operand scales.
// ---------------------------------------------------------------------------
template <int W, int KIN, int DEPTH, int NZT, int WAVES, int SB, class OP>
__global__ void __launch_bounds__(WAVES * 64, 1)
    saa_k_mlp_mfma(MlpDev net, const __bf16* xenc, int64_t N, double* q_out, double* g_out) {
  constexpr int MT = W / 16, KS = W / 32, KS1 = KIN / 32;
  constexpr int MW = MT / WAVES;           // output tiles per wave (SB blocks of 16 samples)
  constexpr int KW = MW / 2;               // k-steps a wave publishes
  constexpr int FB = OP::FB;               // bytes per 16 x 32 fragment
  static_assert(MW % 2 == 0 && KS == KW * WAVES && NZT <= WAVES && SB >= 1 && SB <= 4 && KS1 <= KS,
                "feature split of the width over the waves");
  typedef typename OP::vec vec;
  extern __shared__ uint4 lds[];
  vec* act = (vec*)lds;                                          // [SB][KS][64]: B fragments
  float* smax = (float*)((char*)lds + SB * KS * FB);             // [WAVES][SB][16] (FP8 only)
  constexpr int SMAX = OP::scaled ? WAVES * SB * 16 * 4 : 0;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, g = ln >> 4, c16 = ln & 15;
  _Float16* myg = (_Float16*)((char*)lds + SB * KS * FB + SMAX) + (size_t)wv * DEPTH * MW * SB * 256;
  float* qs = (float*)lds;                                       // [MT][SB][16] (reuses act)
  const int64_t base = (int64_t)blockIdx.x * (16 * SB);
  f32x4 acc[MW][SB];
  int axe[SB];                           // FP8: exponent of the current B operands' scale, per sample block
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) axe[sb] = 0;
  // operand k of the stream in this format (the FP8 copy has 512-byte fragments)
  auto operand = [&](const void* bf16_op) -> const char* {
    if constexpr (OP::scaled)
      return (const char*)net.ws8 + ((const char*)bf16_op - (const char*)net.ws) / 2;
    else
      return (const char*)bf16_op;
  };

  // E8M0 scales that undo the FP8 scalings: operand `op` of the weight
  // stream (A), and the activations of sample block sb (B)
  auto a_scale = [&](int op) -> int {
    int e;
    (void)frexpf(net.wsc_inv[op], &e);   // wsc_inv = 2^(e - 1)
    return 126 + e;
  };
  auto b_scale = [&](int sb) -> int { return 127 - axe[sb]; };
  // B operand of the 16 x 16 x 128 MFMA: this lane's bytes of blocks 4 k4 .. 4 k4 + 3
  auto b_quad = [&](int sb, int k4) -> i32x8 {
    const long* a8 = (const long*)act + (sb * KS + 4 * k4) * 64 + ln;
    const i64x4 v = {a8[0], a8[64], a8[128], a8[192]};
    return __builtin_bit_cast(i32x8, v);
  };

  // Whole-product prefetch (when a product's A fragments fit in 64 VGPRs and
  // a wave may hold 256):
  // the fragments of the next product are loaded while the current one
  // finishes, so their L2 latency hides behind the epilogue and the barriers.
  constexpr int KX = OP::scaled ? KS / 4 : KS;             // MFMA k-steps of a full product
  constexpr int FX = OP::scaled ? 4 * FB : FB;             // bytes per MFMA A fragment
  typedef typename std::conditional<OP::scaled, i32x8, vec>::type avec;
  constexpr bool WHOLE = KX * MW * (int)sizeof(avec) <= 64 * 4 && WAVES <= 8;
  avec ab[WHOLE ? KX : 1][MW];
  auto load_all = [&](const char* A, int mtx, int nks) {
    if constexpr (WHOLE) {
      const char* Aw = A + (size_t)(MW * wv) * FX + ln * (FX / 64);
      const int nkx = OP::scaled ? nks / 4 : nks;
#pragma unroll
      for (int kx = 0; kx < KX; ++kx)
        if (kx < nkx)
#pragma unroll
          for (int j = 0; j < MW; ++j) ab[kx][j] = *(const avec*)(Aw + (size_t)(kx * mtx + j) * FX);
    }
  };

  // acc += A(MW wv + j, ks) B(sb, ks); A fragment (ks, mt) of an operand with
  // mtx row tiles at A + (ks mtx + mt) FB bytes; B from act, or (BF16) from
  // the encoded input for layer 0.  FP8: 16 x 128 fragments (k4, mt) at
  // A + (k4 mtx + mt) 4 FB bytes; `op` is the operand's index in the stream.
  // WHOLE: the A fragments are already in ab (load_all).
  auto product = [&](const char* A, int mtx, int nks, bool from_input, int op) {
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc[j][sb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (WHOLE) {
      int sa = 0, sbv[SB];
      if constexpr (OP::scaled) {
        sa = a_scale(op);
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) sbv[sb] = b_scale(sb);
      }
      const int nkx = OP::scaled ? nks / 4 : nks;
#pragma unroll
      for (int kx = 0; kx < KX; ++kx) {
        if (kx < nkx) {
          avec b[SB];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) {
            if constexpr (OP::scaled) {
              b[sb] = b_quad(sb, kx);
            } else if (from_input) {
              const int64_t smp = base + 16 * sb + c16;
              b[sb] = vec{};
              if (smp < N) b[sb] = *(const vec*)(xenc + smp * KIN + 32 * kx + 8 * g);
            } else {
              b[sb] = act[(sb * KS + kx) * 64 + ln];
            }
          }
#pragma unroll
          for (int j = 0; j < MW; ++j)
#pragma unroll
            for (int sb = 0; sb < SB; ++sb) {
              if constexpr (OP::scaled)
                acc[j][sb] = OP::mma4(ab[kx][j], b[sb], acc[j][sb], sa, sbv[sb]);
              else
                acc[j][sb] = OP::mma(ab[kx][j], b[sb], acc[j][sb]);
            }
        }
      }
    } else if constexpr (OP::scaled) {
      constexpr int KS4 = KS / 4;
      const int nk4 = nks / 4;
      const int sa = a_scale(op);
      int sbv[SB];
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) sbv[sb] = b_scale(sb);
      const char* Aw = A + (size_t)(MW * wv) * (4 * FB) + ln * 32;
      i32x8 a[2][MW];
#pragma unroll
      for (int j = 0; j < MW; ++j) a[0][j] = *(const i32x8*)(Aw + (size_t)j * (4 * FB));
#pragma unroll
      for (int k4 = 0; k4 < KS4; ++k4) {
        if (k4 < nk4) {
          if (k4 + 1 < nk4) {
#pragma unroll
            for (int j = 0; j < MW; ++j)
              a[(k4 + 1) & 1][j] = *(const i32x8*)(Aw + (size_t)((k4 + 1) * mtx + j) * (4 * FB));
          }
          i32x8 b[SB];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) b[sb] = b_quad(sb, k4);
#pragma unroll
          for (int j = 0; j < MW; ++j)
#pragma unroll
            for (int sb = 0; sb < SB; ++sb) acc[j][sb] = OP::mma4(a[k4 & 1][j], b[sb], acc[j][sb], sa, sbv[sb]);
        }
      }
    } else {
      const char* Aw = A + (size_t)(MW * wv) * FB + ln * (FB / 64);
      vec a[3][MW];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int j = 0; j < MW; ++j)
          if (p < nks) a[p][j] = *(const vec*)(Aw + (size_t)(p * mtx + j) * FB);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        if (ks < nks) {
          if (ks + 2 < nks) {
#pragma unroll
            for (int j = 0; j < MW; ++j) a[(ks + 2) % 3][j] = *(const vec*)(Aw + (size_t)((ks + 2) * mtx + j) * FB);
          }
          vec b[SB];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) {
            if (!OP::scaled && from_input) {
              const int64_t smp = base + 16 * sb + c16;
              b[sb] = vec{};
              if (smp < N) b[sb] = *(const vec*)(xenc + smp * KIN + 32 * ks + 8 * g);
            } else {
              b[sb] = act[(sb * KS + ks) * 64 + ln];
            }
          }
#pragma unroll
          for (int j = 0; j < MW; ++j)
#pragma unroll
            for (int sb = 0; sb < SB; ++sb) acc[j][sb] = OP::mma(a[ks % 3][j], b[sb], acc[j][sb]);
        }
      }
    }
  };
  // publish this wave's outputs (acc holds them) as B fragments of k-steps KW wv ..
  auto publish = [&]() {
    if constexpr (OP::scaled) {   // per-sample maxima of this wave's features
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        float m = 0.0f;
#pragma unroll
        for (int j = 0; j < MW; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(acc[j][sb][r]));
        m = fmaxf(m, __shfl_xor(m, 16, 64));
        m = fmaxf(m, __shfl_xor(m, 32, 64));
        if (g == 0) smax[(wv * SB + sb) * 16 + c16] = m;
      }
    }
    __syncthreads();   // every wave finished reading act (and posted its maxima)
    if constexpr (OP::scaled) {
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        float m = 0.0f;
        for (int w = 0; w < WAVES; ++w) m = fmaxf(m, smax[(w * SB + sb) * 16 + c16]);
        axe[sb] = pow2_exp256(m);
      }
    }
#pragma unroll
    for (int jp = 0; jp < KW; ++jp)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        const float e[8] = {acc[2 * jp][sb][0],     acc[2 * jp][sb][1],     acc[2 * jp][sb][2],
                            acc[2 * jp][sb][3],     acc[2 * jp + 1][sb][0], acc[2 * jp + 1][sb][1],
                            acc[2 * jp + 1][sb][2], acc[2 * jp + 1][sb][3]};
        act[(sb * KS + KW * wv + jp) * 64 + ln] = OP::pack(e, ldexpf(1.0f, axe[sb]));
      }
    __syncthreads();
  };

  load_all(operand(net.wp[0]), MT, KS1);
  if constexpr (OP::scaled) {   // FP8: scale and publish the encoded input like a layer output
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) acc[j][sb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // wave w holds input features of k-steps KW w .. (zero beyond KIN)
#pragma unroll
    for (int jp = 0; jp < KW; ++jp) {
      const int ks = KW * wv + jp;
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        const int64_t smp = base + 16 * sb + c16;
        if (ks < KS1 && smp < N) {
          const bf16x8 x = *(const bf16x8*)(xenc + smp * KIN + 32 * ks + 8 * g);
#pragma unroll
          for (int t = 0; t < 8; ++t) acc[2 * jp + t / 4][sb][t % 4] = (float)x[t];
        }
      }
    }
    publish();
  }

  // forward through the hidden layers
#pragma unroll
  for (int L = 0; L < DEPTH; ++L) {
    const float* bl = (L == 0) ? net.b0eff : net.bias[L];
    float4 bias4[MW];   // loaded before the next product's fragments, so waiting for them does not wait for those
#pragma unroll
    for (int j = 0; j < MW; ++j) bias4[j] = *(const float4*)(bl + 16 * (MW * wv + j) + 4 * g);
    product(operand(net.wp[L]), MT, L == 0 ? KS1 : KS, L == 0, L);
    load_all(operand(net.wp[L + 1]), MT, KS);
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      const float4 b4 = bias4[j];
      const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        f16x4 d4;
        float av[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) av[r] = acc[j][sb][r] + bb[r];
        float hv[4];
        _Float16 dv[4];
        gelu_pair2(av[0], av[1], hv[0], hv[1], dv[0], dv[1]);
        gelu_pair2(av[2], av[3], hv[2], hv[3], dv[2], dv[3]);
        d4 = f16x4{dv[0], dv[1], dv[2], dv[3]};
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[j][sb][r] = hv[r];
        *(f16x4*)(myg + (((L * MW + j) * SB + sb) * 64 + ln) * 4) = d4;
      }
    }
    publish();
  }
  // output layer phi = W h + b (rows padded to W), reduced QoI and its gradient
  {
    float4 bias4[MW];
#pragma unroll
    for (int j = 0; j < MW; ++j) bias4[j] = *(const float4*)(net.bc + 16 * (MW * wv + j) + 4 * g);
    product(operand(net.wp[DEPTH]), MT, KS, false, DEPTH);
    load_all(operand(net.wt[DEPTH]), MT, KS);
    // |phi + c|^2 as per-tile partial sums (16 features: a lane's 4 rows,
    // then across the 4 row groups), added in tile order by one wave, so the
    // result does not depend on how the tiles are split over the waves
    float qp[MW][SB];
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      // rows past r_u have zero weights and zero bias + c, so v = 0 there
      const float4 b4 = bias4[j];
      const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        qp[j][sb] = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float v = acc[j][sb][r] + bb[r];
          qp[j][sb] += v * v;
          acc[j][sb][r] = 2.0f * v;
        }
        qp[j][sb] += __shfl_xor(qp[j][sb], 16, 64);
        qp[j][sb] += __shfl_xor(qp[j][sb], 32, 64);
      }
    }
    __syncthreads();   // every wave finished reading act: reuse it for the partial sums [MT][SB][16]
    if (g == 0)
#pragma unroll
      for (int j = 0; j < MW; ++j)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) qs[((MW * wv + j) * SB + sb) * 16 + c16] = qp[j][sb];
    __syncthreads();
    if (wv == 0 && ln < 16 * SB) {
      const int sb = ln >> 4;
      const int64_t smp = base + ln;
      float qsum = 0.0f;
      for (int t = 0; t < MT; ++t) qsum += qs[(t * SB + sb) * 16 + c16];
      if (smp < N) q_out[smp] = (double)qsum + net.c0;
    }
    publish();
  }
  // reverse pass: delta h_{L-1} = W_L^T delta a_L; delta a_{L-1} = GELU'(a_{L-1}) delta h_{L-1}
#pragma unroll
  for (int L = DEPTH; L >= 1; --L) {
    product(operand(net.wt[L]), MT, KS, false, DEPTH + 1 + (DEPTH - L));
    if (L > 1) load_all(operand(net.wt[L - 1]), MT, KS);
#pragma unroll
    for (int j = 0; j < MW; ++j)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb) {
        const f16x4 d4 = *(const f16x4*)(myg + ((((L - 1) * MW + j) * SB + sb) * 64 + ln) * 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[j][sb][r] *= (float)d4[r];
      }
    publish();
  }
  // dq/dz = W_0[:, r_m:]^T delta a_0: NZT row tiles, one per wave (waves >= NZT idle)
  if (wv < NZT) {
    f32x4 az[SB];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) az[sb] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (OP::scaled) {
      const char* Aw = operand(net.w0z) + (size_t)wv * (4 * FB) + ln * 32;
      const int sa = a_scale(2 * DEPTH + 1);
#pragma unroll
      for (int k4 = 0; k4 < KS / 4; ++k4) {
        const i32x8 a = *(const i32x8*)(Aw + (size_t)(k4 * NZT) * (4 * FB));
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) az[sb] = OP::mma4(a, b_quad(sb, k4), az[sb], sa, b_scale(sb));
      }
    } else {
      const char* Aw = operand(net.w0z) + (size_t)wv * FB + ln * (FB / 64);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const vec a = *(const vec*)(Aw + (size_t)(ks * NZT) * FB);
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) az[sb] = OP::mma(a, act[(sb * KS + ks) * 64 + ln], az[sb]);
      }
    }
    const int d_z = net.d_z;
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t smp = base + 16 * sb + c16;
      if (smp < N)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int zi = 16 * wv + 4 * g + r;
          if (zi < d_z) g_out[smp * d_z + zi] = (double)az[sb][r];
        }
    }
  }
}

// FP8 copy of the BF16 weights: every operand scaled by its own power of
// two (largest magnitude -> [112, 224)).  Operand k spans 16 x 32 blocks
// [off[k], off[k + 1]) of the BF16 stream, with mtx[k] row tiles; one
// workgroup per operand finds its scale.
struct OpRanges {
  int n;
  int64_t off[2 * MLP_MAX_DEPTH + 3];
  int mtx[2 * MLP_MAX_DEPTH + 2];
};

__global__ void __launch_bounds__(256) saa_k_op_scale(const __bf16* ws, OpRanges ops, float* wsc_inv) {
  __shared__ float red[4];
  const int k = blockIdx.x;
  const int64_t e0 = ops.off[k] * 512, e1 = ops.off[k + 1] * 512;
  float m = 0.0f;
  for (int64_t i = e0 + threadIdx.x; i < e1; i += 256) m = fmaxf(m, fabsf((float)ws[i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    wsc_inv[k] = 1.0f / pow2_scale(m, 224.0f);
  }
}

// The FP8 stream holds each operand in 16 x 128 fragments (k4, mt) of 2 KB
// at (k4 mtx + mt) 2 KB from the operand's start (the same start as in
// 512-byte blocks): lane l's 32 bytes are its 8 values of the 16 x 32 blocks
// (4 k4 + t, mt), t = 0..3, in order.  Four bytes per thread.
__global__ void saa_k_pack_fp8(const __bf16* ws, OpRanges ops, const float* wsc_inv, int64_t n, uint8_t* dst) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (t >= n) return;
  const int64_t f = t / 512;
  int k = 0;
  while (k + 1 < ops.n && ops.off[k + 1] <= f) ++k;
  const int64_t rel = t - ops.off[k] * 512;
  const int64_t F = rel / 2048;
  const int within = (int)(rel % 2048), lane = within / 32, byte = within % 32;
  const int64_t k4 = F / ops.mtx[k], mt = F % ops.mtx[k];
  const int64_t src = (ops.off[k] + (4 * k4 + byte / 8) * ops.mtx[k] + mt) * 512 + lane * 8 + byte % 8;
  const float sc = 1.0f / wsc_inv[k];
  int v = 0;
  v = __builtin_amdgcn_cvt_pk_fp8_f32((float)ws[src] * sc, (float)ws[src + 1] * sc, v, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32((float)ws[src + 2] * sc, (float)ws[src + 3] * sc, v, true);
  *(int*)(dst + t) = v;
}

// ---------------------------------------------------------------------------
// FP32 reference kernel (plain FMA): one wave carries 2 samples; each lane
// owns output features lane, lane + 64, ...; activations in LDS.
// ---------------------------------------------------------------------------
template <int W, int DEPTH>
__global__ void __launch_bounds__(256) saa_k_mlp_fp32(MlpDev net, const double* xi, int nkl, const int* order,
                                                      int64_t N, double* q_out, double* g_out) {
  constexpr int S = 2;          // samples per wave
  constexpr int J = W / 64;     // outputs per lane
  __shared__ float hbuf[4][S][W];
  __shared__ float dg[4][DEPTH][S][W];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int r_m = net.r_m, r_u = net.r_u, d_z = net.d_z;
  const int64_t s0 = ((int64_t)blockIdx.x * 4 + wv) * S;   // waves past N compute on zeros
  float (*h)[W] = hbuf[wv];
  for (int si = 0; si < S; ++si)
    for (int k = ln; k < W; k += 64) {
      const int64_t s = s0 + si;
      h[si][k] = (s < N && k < r_m) ? (float)xi[s * nkl + order[k]] : 0.0f;
    }
  __syncthreads();
  for (int L = 0; L <= DEPTH; ++L) {
    const int kin = (L == 0) ? r_m : W;
    const int rows = (L == DEPTH) ? r_u : W;
    const float* wt = net.wtn[L];   // kin_L x rows (transposed natural), contiguous in output
    float a[S][J];
    for (int si = 0; si < S; ++si)
      for (int j = 0; j < J; ++j) a[si][j] = 0.0f;
    for (int k = 0; k < kin; ++k) {
      float wk[J];
      for (int j = 0; j < J; ++j) {
        const int m = ln + 64 * j;
        wk[j] = (m < rows) ? wt[(int64_t)k * rows + m] : 0.0f;
      }
      for (int si = 0; si < S; ++si) {
        const float hk = h[si][k];
        for (int j = 0; j < J; ++j) a[si][j] += wk[j] * hk;
      }
    }
    __syncthreads();
    for (int si = 0; si < S; ++si)
      for (int j = 0; j < J; ++j) {
        const int m = ln + 64 * j;
        const float b = (L == 0) ? net.b0eff[m] : net.bias[L][m];
        const float v = a[si][j] + b;
        if (L < DEPTH) {
          dg[wv][L][si][m] = dgelu_f(v);
          h[si][m] = gelu_f(v);
        } else {
          h[si][m] = (m < r_u) ? v + net.c[m] : 0.0f;   // phi + c
        }
      }
    __syncthreads();
  }
  // q and delta = 2 (phi + c)
  for (int si = 0; si < S; ++si) {
    float qs = 0.0f;
    for (int m = ln; m < W; m += 64) qs += h[si][m] * h[si][m];
    qs = wave_sum(qs);
    const int64_t s = s0 + si;
    if (ln == 0 && s < N) q_out[s] = (double)qs + net.c0;
  }
  __syncthreads();
  for (int si = 0; si < S; ++si)
    for (int m = ln; m < W; m += 64) h[si][m] *= 2.0f;
  __syncthreads();
  // reverse: dh_{L-1}[k] = sum_m W_L[m][k] da_L[m]
  for (int L = DEPTH; L >= 1; --L) {
    const int rows = (L == DEPTH) ? r_u : W;
    const float* w = net.wn[L];   // rows x W natural
    float a[S][J];
    for (int si = 0; si < S; ++si)
      for (int j = 0; j < J; ++j) a[si][j] = 0.0f;
    for (int m = 0; m < rows; ++m) {
      float wk[J];
      for (int j = 0; j < J; ++j) wk[j] = w[(int64_t)m * W + ln + 64 * j];
      for (int si = 0; si < S; ++si) {
        const float dm = h[si][m];
        for (int j = 0; j < J; ++j) a[si][j] += wk[j] * dm;
      }
    }
    __syncthreads();
    for (int si = 0; si < S; ++si)
      for (int j = 0; j < J; ++j) {
        const int k = ln + 64 * j;
        h[si][k] = a[si][j] * dg[wv][L - 1][si][k];
      }
    __syncthreads();
  }
  // dq/dz_i = sum_m W_0[m][r_m + i] da_0[m]
  const float* w0 = net.wn[0];
  for (int si = 0; si < S; ++si) {
    const int64_t s = s0 + si;
    for (int zi = ln; zi < d_z; zi += 64) {
      float acc = 0.0f;
      for (int m = 0; m < W; ++m) acc += w0[(int64_t)m * (r_m + d_z) + r_m + zi] * h[si][m];
      if (s < N) g_out[s * d_z + zi] = (double)acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace saa_launch {

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void mlp_pack_fwd(void* dst, const float* src, int rows, int cols, int src_rows, int src_cols, int src_ld,
                  int natural, hipStream_t st) {
  saa_k_pack_fwd<<<nblk((int64_t)rows * cols, 256), 256, 0, st>>>((__bf16*)dst, src, rows, cols, src_rows,
                                                                  src_cols, src_ld, natural);
}
void mlp_pack_bwd(void* dst, const float* src, int rows, int cols, int src_rows, int src_cols, int src_ld,
                  int col0, hipStream_t st) {
  saa_k_pack_bwd<<<nblk((int64_t)rows * cols, 256), 256, 0, st>>>((__bf16*)dst, src, rows, cols, src_rows,
                                                                  src_cols, src_ld, col0);
}
void mlp_transpose(float* dst, const float* src, int rows, int cols, int src_ld, hipStream_t st) {
  saa_k_transpose<<<nblk((int64_t)rows * cols, 256), 256, 0, st>>>(dst, src, rows, cols, src_ld);
}
void mlp_pad(float* dst, const float* src, int n_src, int n_dst, hipStream_t st) {
  saa_k_pad<<<nblk(n_dst, 256), 256, 0, st>>>(dst, src, n_src, n_dst);
}
void mlp_encode(const double* xi, int nkl, const int* order, int r_m, int kin, int64_t N, void* X, hipStream_t st) {
  saa_k_encode<<<nblk(N * kin, 256), 256, 0, st>>>(xi, nkl, order, r_m, kin, N, (__bf16*)X);
}
void mlp_add_pad(float* dst, const float* a, const float* b, int n, int w, hipStream_t st) {
  saa_k_add_pad<<<nblk(w, 256), 256, 0, st>>>(dst, a, b, n, w);
}
void mlp_b0eff(float* b0eff, const float* W0zT, const float* b0, const double* z, int width, int d_z,
               hipStream_t st) {
  saa_k_b0eff<<<nblk(width, 64), 64, 0, st>>>(b0eff, W0zT, b0, z, width, d_z);
}

// Network shapes of the fused kernel (and of the FP32 reference kernel):
// width 256 (r_m <= 128, d_z <= 32, 64 samples per 8-wave workgroup) or
// width 512 (r_m <= 256, d_z <= 64, 32 samples per workgroup: the fp16
// GELU' of 4 layers x 512 features x 32 samples fills 128 KB of LDS), depth
// 4, r_u <= width.  prec: 0 FP32 reference kernel, 1 BF16, 2 FP8.
// Tile shapes of the fused kernel (the autotuner's candidates): waves per
// workgroup x samples per workgroup.  Every shape computes each output of
// each product with the same k order, so all give bitwise the same results.
template <int W_, int KIN_, int NZT_, int WAVES_, int SB_>
struct MlpShape {
  static constexpr int W = W_, KIN = KIN_, NZT = NZT_, WAVES = WAVES_, SB = SB_;
};
int mlp_kin(int width) { return width == 512 ? 256 : 128; }
int mlp_nzt(int width) { return width == 512 ? 4 : 2; }
int mlp_variants(int width) { return width == 512 ? 2 : 3; }
bool mlp_shape_ok(int width, int depth, int r_m, int d_z, int r_u) {
  if (depth != 4 || r_m < 1 || d_z < 1 || r_u < 1 || r_u > width) return false;
  if (width == 256) return r_m <= 128 && d_z <= 32;
  if (width == 512) return r_m <= 256 && d_z <= 64;
  return false;
}

template <class OP, class SH>
static int mlp_launch(const MlpDev& net, const void* xenc, int64_t N, double* q, double* g, hipStream_t st) {
  const void* fn = (const void*)saa_k_mlp_mfma<SH::W, SH::KIN, 4, SH::NZT, SH::WAVES, SH::SB, OP>;
  const size_t gelu_lds = (size_t)4 * SH::W * 2 * 16 * SH::SB;   // DEPTH x width x fp16 x samples
  const size_t lds =
      (size_t)SH::SB * (SH::W / 32) * OP::FB + (OP::scaled ? SH::WAVES * SH::SB * 16 * 4 : 0) + gelu_lds;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -2;
    attr_set = true;
  }
  const unsigned grid = (unsigned)((N + 16 * SH::SB - 1) / (16 * SH::SB));
  saa_k_mlp_mfma<SH::W, SH::KIN, 4, SH::NZT, SH::WAVES, SH::SB, OP>
      <<<grid, SH::WAVES * 64, lds, st>>>(net, (const __bf16*)xenc, N, q, g);
  return 0;
}

// Variant v of the width's candidates: width 256: (8 waves, 64 samples),
// (8, 32), (4, 64); width 512: (8 waves, 32 samples), (16, 32).
template <class OP>
static int mlp_variant(int v, const MlpDev& net, const void* xenc, int64_t N, double* q, double* g, hipStream_t st) {
  if (net.width == 256) {
    if (v == 1) return mlp_launch<OP, MlpShape<256, 128, 2, 8, 2>>(net, xenc, N, q, g, st);
    if (v == 2) return mlp_launch<OP, MlpShape<256, 128, 2, 4, 4>>(net, xenc, N, q, g, st);
    return mlp_launch<OP, MlpShape<256, 128, 2, 8, 4>>(net, xenc, N, q, g, st);
  }
  if (v == 1) return mlp_launch<OP, MlpShape<512, 256, 4, 16, 2>>(net, xenc, N, q, g, st);
  return mlp_launch<OP, MlpShape<512, 256, 4, 8, 2>>(net, xenc, N, q, g, st);
}

// The autotuner's key of a launch: width, precision and N rounded up to a
// power of two.
std::string mlp_tune_key(int width, int prec, int64_t N) {
  int64_t b = 1;
  while (b < N) b <<= 1;
  return "mlp/w" + std::to_string(width) + "/p" + std::to_string(prec) + "/N" + std::to_string(b);
}

int mlp_eval(const MlpDev& net, int prec, const double* xi, int nkl, const int* order, const void* xenc,
             int64_t N, double* q, double* g, int n_cu, hipStream_t st) {
  if (!mlp_shape_ok(net.width, net.depth, net.r_m, net.d_z, net.r_u)) return -1;
  (void)n_cu;
  const int W = net.width;
  if (prec == 1 || prec == 2) {
    const int kin = mlp_kin(W), nzt = mlp_nzt(W);
    // wp[0], wp[1..4] and wt[4..1], w0z (the stream of the model's packing)
    const int64_t frags =
        (int64_t)(W / 16) * (kin / 32) + 8 * (int64_t)(W / 16) * (W / 32) + (int64_t)nzt * (W / 32);
    if (net.kin != kin || net.ws_frags != frags) return -1;
    if (prec == 2 && (!net.ws8 || !net.wsc_inv)) return -1;
    auto run = [&](int v) {
      return prec == 1 ? mlp_variant<OpBF16>(v, net, xenc, N, q, g, st)
                       : mlp_variant<OpFP8>(v, net, xenc, N, q, g, st);
    };
    const std::string key = mlp_tune_key(W, prec, N);
    int v = saa_tune::lookup(key);
    if (v < 0 || v >= mlp_variants(W)) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return run(0);   // no timing under capture: the default shape
      }
      // time every candidate once (the launches are idempotent: q and g are
      // rewritten), keep the fastest, and run it last so its outputs stay
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -2;
      float best = INFINITY;
      int pick = 0;
      for (int c = 0; c < mlp_variants(W); ++c) {
        int rc = run(c);   // warm (LDS attribute, code object)
        if (!rc && hipEventRecord(e0, st) == hipSuccess) rc = run(c);
        float ms = INFINITY;
        if (!rc && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess)
          (void)hipEventElapsedTime(&ms, e0, e1);
        if (!rc && ms < best) {
          best = ms;
          pick = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      saa_tune::store(key, pick);
      v = pick;
    }
    return run(v);
  }
  const int64_t blocks = (N + 7) / 8;
  if (W == 256) saa_k_mlp_fp32<256, 4><<<(unsigned)blocks, 256, 0, st>>>(net, xi, nkl, order, N, q, g);
  else saa_k_mlp_fp32<512, 4><<<(unsigned)blocks, 256, 0, st>>>(net, xi, nkl, order, N, q, g);
  return 0;
}

// FP8 weight stream and per-operand scales from the BF16 stream (operands
// in stream order wp[0..depth], wt[depth..1], w0z: width / 16 row tiles,
// the last one mlp_nzt(width)).
void mlp_pack_fp8(const void* ws, const int64_t* op_off, int n_ops, int width, float* wsc_inv, void* ws8,
                  int64_t n_frags, hipStream_t st) {
  OpRanges r{};
  r.n = n_ops;
  for (int k = 0; k <= n_ops; ++k) r.off[k] = op_off[k];
  for (int k = 0; k < n_ops; ++k) r.mtx[k] = k + 1 < n_ops ? width / 16 : mlp_nzt(width);
  saa_k_op_scale<<<n_ops, 256, 0, st>>>((const __bf16*)ws, r, wsc_inv);
  const int64_t n = n_frags * 512;
  saa_k_pack_fp8<<<nblk(n / 4, 256), 256, 0, st>>>((const __bf16*)ws, r, wsc_inv, n, (uint8_t*)ws8);
}

}  // namespace saa_launch

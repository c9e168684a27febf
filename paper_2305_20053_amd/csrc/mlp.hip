// MR-DINO surrogate evaluation (paper Sec. 3.3, eq. (rbnet); Sec. 3.1,
// eq. (neural_operator_risk) / (neural_operator_gradient)):
//
//   x = [xi_hat (r_m leading KL coordinates); z]
//   a_L = W_L h_{L-1} + b_L, h_L = GELU(a_L), L = 0..depth-1;  phi = W_depth h + b
//   q = |phi + c|^2 + c0                 (reduced quadratic QoI, Sec. 3.3)
//   dq/dz by reverse mode: delta = 2 (phi + c), back through the layers with
//   GELU'(a_L), and finally the control columns of W_0.
//
// BF16 kernel (MFMA v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Each wave
// carries 16 samples through the whole network.  Products are formed
// transposed, C = W_L * H^T: output features run along the MFMA M dimension and
// samples along N, so one lane holds, for its sample, 4 consecutive features of
// every 16-feature tile.  That accumulator layout is the B-operand layout of the
// next layer up to a fixed permutation inside every 32-feature block
// (slot 8g + t holds feature 4g + t for t < 4 and 16 + 4g + t - 4 for t >= 4);
// the permutation is folded into the stored weight copies, so activations never
// leave registers between layers.  GELU'(a_L) of every layer is kept in LDS as
// fp16 for the reverse pass.
//
// The weights (A operands) reach the MFMAs through LDS: every BF16 fragment of
// every layer is stored once, in the order the kernel consumes it, in one
// "weight stream"; the waves of a workgroup copy it to LDS together, F
// fragments (one stage) at a time, two stages ahead in registers and double
// buffered in LDS, and all of them read their fragments from that shared copy.
// Each weight byte thus crosses L2 once per workgroup instead of once per wave.
#include <hip/hip_fp16.h>

#include "common.h"
#include "mlp.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ int kperm(int k) {
  const int b = k & ~31, kk = k & 31, g = kk >> 3, t = kk & 7;
  return b + (t < 4 ? 4 * g + t : 16 + 4 * g + (t - 4));
}

// GELU and its derivative for the BF16 kernel, branch-free: Phi(a) =
// (1 + erf(a / sqrt 2)) / 2 with erf from Abramowitz & Stegun (1964), formula
// 7.1.26 (absolute error <= 1.5e-7, far below BF16 rounding); the factor
// exp(-a^2 / 2) is shared with GELU'(a) = Phi(a) + a phi(a).
__device__ __forceinline__ void gelu_pair(float a, float& h, float& dh) {
  const float x = fabsf(a) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  const float p =
      t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = __expf(-x * x);
  const float phi2 = 0.5f * copysignf(1.0f - p * e, a) + 0.5f;   // Phi(a)
  h = a * phi2;
  dh = fmaf(a * 0.39894228040143268f, e, phi2);
}

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float dgelu_f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

// Operand formats of the fused kernel.  Both use a 16 x 16 x 32 MFMA with the
// same lane layout (lane 16 g + c: row / column c, k = 8 g .. 8 g + 8):
//  OpBF16: BF16 values, 1 KB per 16 x 32 fragment;
//  OpFP8:  FP8 (E4M3) values, 512 B per fragment.  Weights carry a power-of-two
//          scale per operand, activations one per sample (from the largest
//          magnitude of the sample's 256 features), both undone in FP32 after
//          the product, so only the 3-bit mantissa rounding remains.
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
  __device__ static f32x4 mma(vec a, vec b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
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

// Power of two s with m s in [128, 256) (1 for m = 0): the FP8 operand scale
// of values of largest magnitude m (E4M3 holds magnitudes up to 448).
__device__ __forceinline__ float pow2_scale(float m, float top) {
  if (!(m > 0.0f) || !(m < INFINITY)) return 1.0f;
  int e;
  (void)frexpf(top / m, &e);
  e = e - 1 < -60 ? -60 : (e - 1 > 60 ? 60 : e - 1);
  return ldexpf(1.0f, e);
}

// Weight stream staged through LDS (see the header).  A fragment is 16 rows x
// 32 columns (FB bytes); lane 16 g + c holds row c, columns 8 g .. 8 g + 8.
// The stream holds the fragments of every operand in consumption order:
// operand by operand, and inside one operand k-step by k-step, 16-row tile by
// tile.  Stage s = fragments [s F, (s + 1) F) = one contiguous block.
template <int WAVES, int F, class OP>
struct WStream {
  typedef OP Op;
  static constexpr int FR = F;
  static constexpr int UNITS = F * OP::FB / 16;          // 16-byte units per stage
  static constexpr int PER = UNITS / (WAVES * 64);       // per thread per stage
  static_assert(UNITS % (WAVES * 64) == 0, "a stage splits evenly over the threads");
  const uint4* src;   // the stream
  uint4* buf;         // two LDS stage buffers
  int nst;            // stages in the stream
  int s;              // stage being consumed (held in buf[s & 1])
  uint4 ra[PER];      // stage s + 1
  uint4 rb[PER];      // stage s + 2
  // stages past the end re-read the last one (never published)
  __device__ __forceinline__ void load(uint4 (&r)[PER], int stage) {
    const int64_t b = (int64_t)(stage < nst ? stage : nst - 1) * UNITS + threadIdx.x;
#pragma unroll
    for (int k = 0; k < PER; ++k) r[k] = src[b + k * WAVES * 64];
  }
  __device__ __forceinline__ void store(const uint4 (&r)[PER], int b) {
#pragma unroll
    for (int k = 0; k < PER; ++k) buf[b * UNITS + threadIdx.x + k * WAVES * 64] = r[k];
  }
  __device__ __forceinline__ void begin() {
    load(ra, 0);
    store(ra, 0);
    load(ra, 1);
    load(rb, 2);
    s = 0;
    __syncthreads();
  }
  __device__ __forceinline__ typename OP::vec frag(int j) const {
    const char* b = (const char*)(buf + (s & 1) * UNITS);
    return *(const typename OP::vec*)(b + j * OP::FB + (threadIdx.x & 63) * (OP::FB / 64));
  }
  // End of stage s: publish stage s + 1 (its buffer held stage s - 1, which
  // every wave finished before the previous barrier), then prefetch s + 3.
  __device__ __forceinline__ void advance() {
    store(ra, (s + 1) & 1);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) ra[k] = rb[k];
    load(rb, s + 3);
    ++s;
  }
};

// acc[mt] += A(mt, ks) * hb[ks] for ks < NK, mt < MT, with the A fragments
// taken from the stream in order.
template <int MT, int NK, int KSA, class S, class V>
__device__ __forceinline__ void stream_gemm(S& ws, const V (&hb)[KSA], f32x4 (&acc)[MT]) {
  static_assert((MT * NK) % S::FR == 0, "operands start and end on stage boundaries");
#pragma unroll
  for (int f0 = 0; f0 < MT * NK; f0 += S::FR) {
    // all fragment reads of the stage first, so that their LDS latencies
    // overlap instead of stalling each MFMA
    typename S::Op::vec a[S::FR];
#pragma unroll
    for (int j = 0; j < S::FR; ++j) a[j] = ws.frag(j);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < S::FR; ++j) {
      const int f = f0 + j, ks = f / MT, mt = f % MT;
      acc[mt] = S::Op::mma(a[j], hb[ks], acc[mt]);
    }
    ws.advance();
  }
}

// Operands of the next product from the 64 FP32 values of a lane (4 per
// 16-feature tile; tiles 2 ks, 2 ks + 1 form k-step ks).  Returns the
// per-sample scale applied (1 for unscaled formats).
template <class OP, int MT, int KS>
__device__ __forceinline__ float pack_all(const f32x4 (&v)[MT], typename OP::vec (&hb)[KS]) {
  float sc = 1.0f;
  if constexpr (OP::scaled) {
    float m = 0.0f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(v[mt][r]));
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    sc = pow2_scale(m, 256.0f);
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const float e[8] = {v[2 * ks][0],     v[2 * ks][1],     v[2 * ks][2],     v[2 * ks][3],
                        v[2 * ks + 1][0], v[2 * ks + 1][1], v[2 * ks + 1][2], v[2 * ks + 1][3]};
    hb[ks] = OP::pack(e, sc);
  }
  return sc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Weight packing (after every change of the FP32 master parameters)
// ---------------------------------------------------------------------------

// Position t of a stored rows x cols operand (stream order, see WStream)
// -> logical (row m, column k).
__device__ __forceinline__ void frag_pos(int64_t t, int rows, int& m, int& k) {
  const int e = (int)(t & 7);
  const int ln = (int)((t >> 3) & 63);
  const int64_t f = t >> 9;                // fragment index ks * (rows/16) + mt
  const int nmt = rows >> 4;
  const int ks = (int)(f / nmt), mt = (int)(f % nmt);
  m = 16 * mt + (ln & 15);
  k = 32 * ks + 8 * (ln >> 4) + e;
}

// Forward BF16 operand (stream order): logical [m][k] = W[m][kperm(k)] (or
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

// Backward BF16 operand (stream order): logical [m][k] = W[kperm(k)][col0 + m],
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
// k < r_m, 0 up to 128 (the leading KL coordinates, Sec. 3.3).  The samples
// are fixed, so this runs once per sample set.
__global__ void saa_k_encode(const double* xi, int nkl, const int* order, int r_m, int64_t N, __bf16* X) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * 128) return;
  const int64_t s = t >> 7;
  const int k = (int)(t & 127);
  X[t] = (__bf16)(k < r_m ? (float)xi[s * nkl + order[k]] : 0.0f);
}

// dst[i] = a[i] + b[i] for i < n, 0 for n <= i < w.
__global__ void saa_k_add_pad(float* dst, const float* a, const float* b, int n, int w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < w) dst[i] = i < n ? a[i] + b[i] : 0.0f;
}

// b0eff[f] = b_0[f] + sum_k W_0[f][r_m + k] z_k  (the control enters only
// through the first layer and is shared by all samples).
__global__ void saa_k_b0eff(float* b0eff, const float* W0, const float* b0, const double* z, int width, int r_m,
                            int d_z) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= width) return;
  const float* w = W0 + (int64_t)f * (r_m + d_z) + r_m;
  float acc = b0[f];
#pragma unroll
  for (int k = 0; k < 32; ++k)   // d_z <= 32: every load issued at once
    if (k < d_z) acc += w[k] * (float)z[k];
  b0eff[f] = acc;
}

// ---------------------------------------------------------------------------
// Fused MFMA forward + reverse kernel (BF16 or FP8 operands, FP32 accumulation)
// ---------------------------------------------------------------------------
// Operand index of each product in the weight stream (its scale in net.wsc):
// forward layers 0..DEPTH, reverse layers DEPTH..1 -> DEPTH + 1.., w0z last.
template <int W, int KIN, int DEPTH, int WAVES, int NZT, int F, class OP>
__global__ void __launch_bounds__(WAVES * 64, 1)
    saa_k_mlp_mfma(MlpDev net, const __bf16* xenc, int64_t N, double* q_out, double* g_out) {
  constexpr int MT = W / 16;   // 16-feature tiles of a layer output
  constexpr int KS = W / 32;   // 32-feature k-steps of a layer input
  constexpr int KS1 = KIN / 32;
  typedef WStream<WAVES, F, OP> Stream;
  typedef typename OP::vec vec;
  // LDS: two weight-stream stages, then GELU'(a) as [WAVES][DEPTH][MT][64 lanes][4] fp16
  extern __shared__ uint4 lds[];
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63, g = ln >> 4, c16 = ln & 15;
  _Float16* my = (_Float16*)(lds + 2 * Stream::UNITS) + (size_t)wv * DEPTH * MT * 256;
  Stream ws;
  ws.src = (const uint4*)(OP::scaled ? net.ws8 : net.ws);
  ws.buf = lds;
  ws.nst = net.ws_frags / F;
  ws.begin();
  const int d_z = net.d_z;
  // combined scale of a product: 1 / (weight scale x activation scale)
  auto unscale = [&](int op, float ax) -> float { return OP::scaled ? net.wsc_inv[op] / ax : 1.0f; };

  // one 16 * WAVES-sample tile per workgroup (a persistent loop would let the
  // compiler hoist every bias load out of it and spill)
  {
    const int64_t base = (int64_t)blockIdx.x * (16 * WAVES);
    const int64_t s = base + wv * 16 + c16;
    const bool valid = s < N;
    vec hb[KS];
    f32x4 acc[MT];
    float ax = 1.0f;   // scale of the activations in hb (per sample)
    // encoded input (KIN BF16 per sample, see saa_k_encode)
    if constexpr (OP::scaled) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) {
        bf16x8 x = bf16x8{};
        if (valid) x = *(const bf16x8*)(xenc + s * KIN + 32 * ks + 8 * g);
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[2 * ks + t / 4][t % 4] = (float)x[t];
      }
      ax = pack_all<OP>(acc, hb);
    } else {
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) {
        hb[ks] = vec{};
        if (valid) hb[ks] = *(const vec*)(xenc + s * KIN + 32 * ks + 8 * g);
      }
#pragma unroll
      for (int ks = KS1; ks < KS; ++ks) hb[ks] = vec{};
    }

    // forward through the hidden layers
#pragma unroll
    for (int L = 0; L < DEPTH; ++L) {
      const float* bl = (L == 0) ? net.b0eff : net.bias[L];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (L == 0) stream_gemm<MT, KS1>(ws, hb, acc);
      else stream_gemm<MT, KS>(ws, hb, acc);
      const float cs = unscale(L, ax);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const float4 b4 = *(const float4*)(bl + 16 * mt + 4 * g);
        const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
        f16x4 d4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float h, dh;
          gelu_pair(OP::scaled ? fmaf(acc[mt][r], cs, bb[r]) : acc[mt][r] + bb[r], h, dh);
          d4[r] = (_Float16)dh;
          acc[mt][r] = h;
        }
        *(f16x4*)(my + ((L * MT + mt) * 64 + ln) * 4) = d4;
      }
      ax = pack_all<OP>(acc, hb);
    }
    // output layer phi = W h + b (rows padded to W), reduced QoI and its gradient
    {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      stream_gemm<MT, KS>(ws, hb, acc);
      const float cs = unscale(DEPTH, ax);
      float qs = 0.0f;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        // rows past r_u have zero weights and zero bias + c, so v = 0 there
        const float4 b4 = *(const float4*)(net.bc + 16 * mt + 4 * g);
        const float bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float v = OP::scaled ? fmaf(acc[mt][r], cs, bb[r]) : acc[mt][r] + bb[r];
          qs += v * v;
          acc[mt][r] = 2.0f * v;
        }
      }
      qs += __shfl_xor(qs, 16, 64);
      qs += __shfl_xor(qs, 32, 64);
      if (g == 0 && valid) q_out[s] = (double)qs + net.c0;
      ax = pack_all<OP>(acc, hb);
    }
    // reverse pass: delta h_{L} = W_{L+1}^T delta a_{L+1}; delta a_L = GELU'(a_L) delta h_L
#pragma unroll
    for (int L = DEPTH; L >= 1; --L) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
      stream_gemm<MT, KS>(ws, hb, acc);
      const float cs = unscale(DEPTH + 1 + (DEPTH - L), ax);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const f16x4 d4 = *(const f16x4*)(my + (((L - 1) * MT + mt) * 64 + ln) * 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mt][r] = (OP::scaled ? acc[mt][r] * cs : acc[mt][r]) * (float)d4[r];
      }
      ax = pack_all<OP>(acc, hb);
    }
    // dq/dz = W_0[:, r_m:]^T delta a_0
    {
      f32x4 accz[NZT];
#pragma unroll
      for (int zt = 0; zt < NZT; ++zt) accz[zt] = f32x4{0.f, 0.f, 0.f, 0.f};
      stream_gemm<NZT, KS>(ws, hb, accz);
      const float cs = unscale(2 * DEPTH + 1, ax);
      if (valid) {
#pragma unroll
        for (int zt = 0; zt < NZT; ++zt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int zi = 16 * zt + 4 * g + r;
            if (zi < d_z) g_out[s * d_z + zi] = (double)(OP::scaled ? accz[zt][r] * cs : accz[zt][r]);
          }
      }
    }
  }
}

// FP8 copy of the BF16 weight stream: every operand scaled by its own power of
// two (largest magnitude -> [112, 224)).  Operand k spans fragments
// [off[k], off[k + 1]); one workgroup per operand finds its scale.
struct OpRanges {
  int n;
  int64_t off[2 * MLP_MAX_DEPTH + 3];
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

__global__ void saa_k_pack_fp8(const __bf16* ws, OpRanges ops, const float* wsc_inv, int64_t n, uint8_t* dst) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (t >= n) return;
  const int64_t f = t / 512;
  int k = 0;
  while (k + 1 < ops.n && ops.off[k + 1] <= f) ++k;
  const float sc = 1.0f / wsc_inv[k];
  int v = 0;
  v = __builtin_amdgcn_cvt_pk_fp8_f32((float)ws[t] * sc, (float)ws[t + 1] * sc, v, false);
  v = __builtin_amdgcn_cvt_pk_fp8_f32((float)ws[t + 2] * sc, (float)ws[t + 3] * sc, v, true);
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
void mlp_encode(const double* xi, int nkl, const int* order, int r_m, int64_t N, void* X, hipStream_t st) {
  saa_k_encode<<<nblk(N * 128, 256), 256, 0, st>>>(xi, nkl, order, r_m, N, (__bf16*)X);
}
void mlp_add_pad(float* dst, const float* a, const float* b, int n, int w, hipStream_t st) {
  saa_k_add_pad<<<nblk(w, 256), 256, 0, st>>>(dst, a, b, n, w);
}
void mlp_b0eff(float* b0eff, const float* W0, const float* b0, const double* z, int width, int r_m, int d_z,
               hipStream_t st) {
  saa_k_b0eff<<<nblk(width, 256), 256, 0, st>>>(b0eff, W0, b0, z, width, r_m, d_z);
}

// Supported shapes: width 256, depth 4, r_m <= 128, d_z <= 32.
// prec: 0 FP32 reference kernel, 1 BF16, 2 FP8.
// Supported shapes: width 256, depth 4, r_m <= 128, d_z <= 32.
int mlp_eval(const MlpDev& net, int prec, const double* xi, int nkl, const int* order, const void* xenc,
             int64_t N, double* q, double* g, int n_cu, hipStream_t st) {
  if (net.width != 256 || net.depth != 4 || net.r_m > 128 || net.d_z > 32 || net.r_u > 256) return -1;
  (void)n_cu;
  if (prec == 1 || prec == 2) {
    constexpr int WAVES = 4, F = 16;
    // the stream must hold exactly the operands the kernel consumes
    if (net.kin != 128 || net.ws_frags != 16 * 4 + 4 * 16 * 8 + 4 * 16 * 8 + 2 * 8 || net.ws_frags % F) return -1;
    if (prec == 2 && (!net.ws8 || !net.wsc_inv)) return -1;
    const int64_t tiles = (N + 16 * WAVES - 1) / (16 * WAVES);
    const unsigned grid = (unsigned)tiles;
    const size_t gelu_lds = (size_t)WAVES * 4 * (256 / 16) * 256 * sizeof(_Float16);
    auto run = [&](auto op, const void* fn) -> int {
      typedef decltype(op) OP;
      const size_t lds = 2 * (size_t)F * OP::FB + gelu_lds;
      static bool attr_set[2] = {false, false};
      if (!attr_set[OP::scaled]) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return -2;
        attr_set[OP::scaled] = true;
      }
      saa_k_mlp_mfma<256, 128, 4, WAVES, 2, F, OP><<<grid, WAVES * 64, lds, st>>>(net, (const __bf16*)xenc, N, q, g);
      return 0;
    };
    if (prec == 1) return run(OpBF16{}, (const void*)saa_k_mlp_mfma<256, 128, 4, WAVES, 2, F, OpBF16>);
    return run(OpFP8{}, (const void*)saa_k_mlp_mfma<256, 128, 4, WAVES, 2, F, OpFP8>);
  }
  const int64_t blocks = (N + 7) / 8;
  saa_k_mlp_fp32<256, 4><<<(unsigned)blocks, 256, 0, st>>>(net, xi, nkl, order, N, q, g);
  return 0;
}

// FP8 weight stream and per-operand scales from the BF16 stream.
void mlp_pack_fp8(const void* ws, const int64_t* op_off, int n_ops, float* wsc_inv, void* ws8, int64_t n_frags,
                  hipStream_t st) {
  OpRanges r{};
  r.n = n_ops;
  for (int k = 0; k <= n_ops; ++k) r.off[k] = op_off[k];
  saa_k_op_scale<<<n_ops, 256, 0, st>>>((const __bf16*)ws, r, wsc_inv);
  const int64_t n = n_frags * 512;
  saa_k_pack_fp8<<<nblk(n / 4, 256), 256, 0, st>>>((const __bf16*)ws, r, wsc_inv, n, (uint8_t*)ws8);
}

}  // namespace saa_launch

// The 2D (P1 on the square) and 3D (Q1 on the cube) PDE-form kernels in one
// translation unit, so that a single launch can run samples of problems of
// either dimension: the 3D workload and its 2D companions are solved by one
// state launch and one adjoint launch (the batching across problem sizes of
// the workload; paper Sec. 4.4 motivates serving several configurations
// together).
//
// Workgroups of a mixed launch have 1024 threads (the 2D kernels' size; the
// 3D sample bodies run at that width too).  Workgroup b takes a sample of the
// 3D jobs first (they are the long solves, so they start first), then of the
// 2D jobs: the last job of its kind whose first workgroup is <= b.  The
// dynamic LDS holds the 2D coarse levels when every 2D job keeps them there;
// the 3D bodies use only the static scratch.
#include "pde.hip"
#include "pde3.hip"

template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_state_mixed(const State3Job<TW, TS>* j3, int n3,
                                                        const StateJob<TW, TS>* j2, int n2, SolveParams sp) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  __shared__ double zs[SAA_MAX_DZ];
  __shared__ double Gs[4 * 97];
  const int64_t b = blockIdx.x;
  if (n3 > 0 && (n2 == 0 || b < j2[0].first)) {
    int p = 0;
    for (int k = 1; k < n3; ++k)
      if (b >= j3[k].first) p = k;
    const State3Job<TW, TS>& J = j3[p];
    const int64_t s = b - J.first;
    if (s >= J.N) return;
    state3_sample<TW, TS, BS>(J.g, J.Z, 0, J.k64, J.u, J.f, J.b, sp, J.q, J.newton, J.lin, J.flag, s, red, zs, Gs);
  } else {
    int p = 0;
    for (int k = 1; k < n2; ++k)
      if (b >= j2[k].first) p = k;
    const StateJob<TW, TS>& J = j2[p];
    const int64_t s = b - J.first;
    if (s >= J.N) return;
    state_sample<TW, TS, LDSC>(J.g, J.FT, J.Z, 0, J.em, J.u, J.f, J.b, sp, J.q, J.newton, J.lin, J.flag, s, red, zs);
  }
}

template <typename TW, typename TS, bool LDSC>
__global__ void __launch_bounds__(BS) saa_k_adjoint_mixed(const Adjoint3Job<TW, TS>* j3, int n3,
                                                          const AdjointJob<TW, TS>* j2, int n2, SolveParams sp,
                                                          int act, double act_w) {
  __shared__ double red[SAA_MAX_DZ * (BS / SAA_WAVE)];
  __shared__ double Gs[4 * 97];
  const int64_t b = blockIdx.x;
  if (n3 > 0 && (n2 == 0 || b < j2[0].first)) {
    int p = 0;
    for (int k = 1; k < n3; ++k)
      if (b >= j3[k].first) p = k;
    const Adjoint3Job<TW, TS>& J = j3[p];
    const int64_t s = b - J.first;
    if (s >= J.N) return;
    adjoint3_sample<TW, TS, BS>(J.g, J.k64, J.u, J.bvec, J.lam, J.b, sp, J.q, J.tstar, act, act_w, J.gout, J.lin,
                                J.flag, J.did, s, red, Gs);
  } else {
    int p = 0;
    for (int k = 1; k < n2; ++k)
      if (b >= j2[k].first) p = k;
    const AdjointJob<TW, TS>& J = j2[p];
    const int64_t s = b - J.first;
    if (s >= J.N) return;
    adjoint_sample<TW, TS, LDSC>(J.g, J.FT, J.em, J.u, J.bvec, J.lam, J.b, sp, J.q, J.tstar, act, act_w, J.gout,
                                 J.lin, J.flag, J.did, s, red);
  }
}

namespace saa_launch {

template <typename TW, typename TS>
void state_mixed(const State3Job<TW, TS>* j3, int n3, const StateJob<TW, TS>* j2, int n2, int64_t blocks,
                 size_t lds, const SolveParams& sp, hipStream_t st) {
  if (lds) {
    (void)set_lds_attr((const void*)saa_k_state_mixed<TW, TS, true>, lds);
    saa_k_state_mixed<TW, TS, true><<<(unsigned)blocks, BS, lds, st>>>(j3, n3, j2, n2, sp);
  } else {
    saa_k_state_mixed<TW, TS, false><<<(unsigned)blocks, BS, 0, st>>>(j3, n3, j2, n2, sp);
  }
}

template <typename TW, typename TS>
void adjoint_mixed(const Adjoint3Job<TW, TS>* j3, int n3, const AdjointJob<TW, TS>* j2, int n2, int64_t blocks,
                   size_t lds, const SolveParams& sp, int act, double act_w, hipStream_t st) {
  if (lds) {
    (void)set_lds_attr((const void*)saa_k_adjoint_mixed<TW, TS, true>, lds);
    saa_k_adjoint_mixed<TW, TS, true><<<(unsigned)blocks, BS, lds, st>>>(j3, n3, j2, n2, sp, act, act_w);
  } else {
    saa_k_adjoint_mixed<TW, TS, false><<<(unsigned)blocks, BS, 0, st>>>(j3, n3, j2, n2, sp, act, act_w);
  }
}

#define SAA_INST_MIXED(TW, TS)                                                                                 \
  template void state_mixed<TW, TS>(const State3Job<TW, TS>*, int, const StateJob<TW, TS>*, int, int64_t,    \
                                    size_t, const SolveParams&, hipStream_t);                                 \
  template void adjoint_mixed<TW, TS>(const Adjoint3Job<TW, TS>*, int, const AdjointJob<TW, TS>*, int,         \
                                      int64_t, size_t, const SolveParams&, int, double, hipStream_t);
SAA_INST_MIXED(double, double)
SAA_INST_MIXED(double, float)
SAA_INST_MIXED(float, float)
#undef SAA_INST_MIXED

}  // namespace saa_launch

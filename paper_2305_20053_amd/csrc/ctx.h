// Internal definition of the SAA context, shared by the host runtime files.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/saa.h"
#include "pde.h"
#include "pde3.h"
#include "runtime.h"

namespace saa_rt {

// (M u_target) at the interior nodes (node layout) and u_target^T M u_target
// for a target kind of saa_problem on the n x n mesh.
void target_mass(int n, int target, double u_target, std::vector<double>& mt, double& ctt);

// (M u_target) at the interior nodes and u_target^T M u_target on the
// (n+1)^3 grid (Q1 consistent mass).
void target_mass3(int n, int target, double u_target, std::vector<double>& mt, double& ctt);

// Reduced control Jacobians by adjoints for the states of the last
// saa_solve_states call; JY: device, (N d_Z) x r_u.
int adjoint_jacobians(saa_ctx* c, const saa_options* opt, const double* MPhiT, int r_u, double* JY);

// 3D: control Jacobians du/dz of samples [s0, s0 + ns) for the states of the
// last saa_solve_states call (d_Z linearised solves per sample);
// out (device): ((s - s0) d_Z + k) ld + interior index.
int jacobians3(saa_ctx* c, const saa_options* opt, int64_t s0, int64_t ns, double* out, int64_t ld);

template <typename TS>
struct MgStore {
  DevBuf WE, WN, KD, D, X, B, T, cx, cr, cp, cq;
  bool allocated = false;
  bool built = false;
  MgBufs<TS> view() const {
    MgBufs<TS> m;
    m.WE = (TS*)WE.p;
    m.WN = (TS*)WN.p;
    m.KD = (TS*)KD.p;
    m.D = (TS*)D.p;
    m.X = (TS*)X.p;
    m.B = (TS*)B.p;
    m.T = (TS*)T.p;
    m.cx = (TS*)cx.p;
    m.cr = (TS*)cr.p;
    m.cp = (TS*)cp.p;
    m.cq = (TS*)cq.p;
    return m;
  }
};

template <typename TS>
struct Mg3Store {
  DevBuf E, KD, D, X, B, T, cx, cr, cp, cq;
  bool allocated = false;
  bool built = false;
  Mg3Bufs<TS> view() const {
    Mg3Bufs<TS> m;
    m.E = (TS*)E.p;
    m.KD = (TS*)KD.p;
    m.D = (TS*)D.p;
    m.X = (TS*)X.p;
    m.B = (TS*)B.p;
    m.T = (TS*)T.p;
    m.cx = (TS*)cx.p;
    m.cr = (TS*)cr.p;
    m.cp = (TS*)cp.p;
    m.cq = (TS*)cq.p;
    return m;
  }
};

inline bool is_fin(double x) { return std::isfinite(x); }

// Phase timing with HIP events on the context's stream: marks 0..4 bracket
// [state | reduce 1 | adjoint | reduce 2].
struct PhaseTimer {
  bool on = false;
  hipEvent_t ev[5] = {};
  void mark(hipStream_t st, int k) {
    if (on) (void)hipEventRecord(ev[k], st);
  }
  int create() {
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return SAA_E_DEVICE;
    return SAA_OK;
  }
  ~PhaseTimer() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void ms(double* state, double* adjoint, double* reduce) const {
    float a = 0, b = 0, d = 0, e = 0;
    if (!on) return;
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
    (void)hipEventElapsedTime(&d, ev[2], ev[3]);
    (void)hipEventElapsedTime(&e, ev[3], ev[4]);
    *state = a;
    *reduce = (double)b + e;
    *adjoint = d;
  }
};



}  // namespace saa_rt

constexpr size_t RES_T = 2 + SAA_MAX_DZ;                   // index of t (doubles)
constexpr size_t RES_STATS = sizeof(double) * (RES_T + 1);   // byte offset of the statistics
constexpr size_t RES_BYTES = RES_STATS + sizeof(CvarStats);

// Captured device work of one MR-DINO evaluation (control bias, fused network
// kernel, CVaR reduction) and the arguments baked into it.
struct SurrogateGraph {
  struct Key {
    uint64_t model = 0, version = 0;
    int prec = -1, t_mode = 0;
    double beta = 0, eps = 0, alpha = 0, t_in = 0;
    int64_t N = 0;
    int risk = 0;
    double kappa = 0, tau = 0;
    bool operator==(const Key& o) const {
      return model == o.model && version == o.version && prec == o.prec && t_mode == o.t_mode && beta == o.beta && eps == o.eps &&
             alpha == o.alpha && t_in == o.t_in && N == o.N && risk == o.risk && kappa == o.kappa && tau == o.tau;
    }
  };
  Key key, seen;               // key of `exec`; key of the last eager evaluation
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;   // capture stream (the caller's may be the legacy stream)
  bool disabled = false;       // capture failed once: stay eager
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key = seen = Key{};
  }
  ~SurrogateGraph() {
    reset();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

struct saa_ctx {
  saa_problem prob{};
  int64_t N_max = 0;
  int64_t N = 0;
  hipStream_t st = nullptr;
  PdeGeo geo{};
  bool d3 = false;                    // Q1 on the cube (PDE form only)
  Pde3Geo geo3{};
  saa_rt::DevBuf k64;                 // 3D: fine element kappas in FP64, per sample
  saa_rt::DevBuf G3;                  // 3D: separable source factor table s x (n+1)
  saa_rt::Mg3Store<double> mg3_64;
  saa_rt::Mg3Store<float> mg3_32;
  // 3D threads per sample of the state / adjoint kernels per PDE precision
  // (SAA_FP64, SAA_FP32, SAA_FP32_DC64); 0: chosen by timing at the next call
  int bs3_state[3] = {0, 0, 0};
  int bs3_adj[3] = {0, 0, 0};
  int K1 = 0, dz = 0;
  int64_t n_kl = 0;                   // K1^dim KL coefficients per sample
  int64_t nodes = 0, d_u = 0;
  saa_rt::DevBuf FT, S, amp, em, xi, kap;
  saa_rt::DevBuf src1;   // 2D: the 1D Gaussian factors of the separable source matrix
  saa_rt::DevBuf mt;                  // (M u_target) at interior nodes (node layout), FP64
  std::vector<double> mt_host;        // the same on the host
  double ctt = 0.0;                   // u_target^T M u_target
  int64_t kstride = 0, kchunk = 0;
  saa_rt::MgStore<double> mg64;
  saa_rt::MgStore<float> mg32;
  saa_rt::DevBuf u, f, lam;   // PDE-form node vectors (sized for float64; allocated at first use)
  saa_rt::DevBuf q, g, newton, lin, lin_adj, flag, did, zdev;
  // Results of one call, contiguous so that one copy brings them to the host:
  // doubles [0] J, [1] dJ/dt, [2, 2 + d_Z) grad, [2 + SAA_MAX_DZ] t, then the
  // solver statistics (CvarStats) at byte RES_STATS.
  saa_rt::DevBuf res;
  saa_rt::HostBuf hres;       // pinned host copy of `res`
  saa_rt::DevBuf jobs;        // job tables of multi-problem launches led by this context
  saa_rt::DevBuf cwork;       // CVaR reduction workspace (partials, probe histograms, active set)
  saa_rt::DevBuf enc;         // surrogate input: leading KL coordinates as BF16, N_max x kin
  int enc_rm = -1;            // enc_key(r_m, kin) of what `enc` holds for the installed samples (-1: stale)
  saa_rt::DevBuf order;       // KL modes by increasing |k|^2 (ties lexicographic), K1^dim entries
  saa_rt::PhaseTimer timer;
  saa_ctx* holdout = nullptr;  // held-out samples for the surrogate error estimate (not owned)
  bool poison = false;         // fill the per-call workspaces with NaN before each call (SAA_POISON_WORKSPACE)
  SurrogateGraph sg;
  // The replayed surrogate graph reads z from, and writes its result block
  // to, pinned host memory (hz, hres): no copies around the replay.  While it
  // is captured these point there; otherwise they are null and the device
  // buffers zdev, res are used.
  saa_rt::HostBuf hz;         // pinned host copy of z for the graph (SAA_MAX_DZ doubles)
  const double* z_over = nullptr;
  void* res_over = nullptr;
  const double* zd() const { return z_over ? z_over : (const double*)zdev.p; }
  char* resb() { return (char*)(res_over ? res_over : res.p); }
  double* out() { return (double*)resb(); }
  double* tstar() { return (double*)resb() + RES_T; }
  void* stats() { return resb() + RES_STATS; }
};

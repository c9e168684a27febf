// MR-DINO model object: parameters, packed device operands, evaluation.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ctx.h"
#include "mlp.h"
#include "model.h"

namespace saa_launch {
void mlp_pack_fwd(void* dst, const float* src, int rows, int cols, int src_rows, int src_cols, int src_ld,
                  int natural, hipStream_t st);
void mlp_pack_bwd(void* dst, const float* src, int rows, int cols, int src_rows, int src_cols, int src_ld,
                  int col0, hipStream_t st);
void mlp_transpose(float* dst, const float* src, int rows, int cols, int src_ld, hipStream_t st);
void mlp_pad(float* dst, const float* src, int n_src, int n_dst, hipStream_t st);
void mlp_b0eff(float* b0eff, const float* W0zT, const float* b0, const double* z, int width, int d_z,
               hipStream_t st);
int mlp_eval(const MlpDev& net, int prec, const double* xi, int nkl, const int* order, const void* xenc,
             int64_t N, double* q, double* g, int n_cu, hipStream_t st);
void mlp_pack_fp8(const void* ws, const int64_t* op_off, int n_ops, int width, float* wsc_inv, void* ws8,
                  int64_t n_frags,
                  hipStream_t st);
void mlp_encode(const double* xi, int nkl, const int* order, int r_m, int kin, int64_t N, void* X, hipStream_t st);
int mlp_kin(int width);
int mlp_nzt(int width);
bool mlp_shape_ok(int width, int depth, int r_m, int d_z, int r_u);
void mlp_add_pad(float* dst, const float* a, const float* b, int n, int w, hipStream_t st);
}  // namespace saa_launch

using namespace saa_rt;

namespace saa_model {

int64_t param_count(const mrdino_dims& d) {
  int64_t n = 0;
  int in = d.r_m + d.d_z;
  for (int L = 0; L <= d.depth; ++L) {
    const int out = (L == d.depth) ? d.r_u : d.width;
    n += (int64_t)out * in + out;
    in = out;
  }
  return n;
}

bool dims_supported(const mrdino_dims& d) {
  return saa_launch::mlp_shape_ok(d.width, d.depth, d.r_m, d.d_z, d.r_u);
}

MlpDev view(const mrdino_model* m) {
  MlpDev v{};
  const mrdino_dims& d = m->dims;
  v.r_m = d.r_m;
  v.d_z = d.d_z;
  v.r_u = d.r_u;
  v.width = d.width;
  v.depth = d.depth;
  v.kin = m->kin;
  v.master = (const float*)m->master.p;
  for (int L = 0; L <= d.depth; ++L) {
    v.off_w[L] = m->off_w[L];
    v.off_b[L] = m->off_b[L];
    v.wp[L] = (const char*)m->ws.p + 1024 * m->f_wp[L];
    v.wt[L] = (const char*)m->ws.p + 1024 * m->f_wt[L];
    v.bias[L] = (const float*)m->bias[L].p;
    v.wn[L] = (const float*)m->master.p + m->off_w[L];
    v.wtn[L] = (const float*)m->wtn[L].p;
  }
  v.w0z = (const char*)m->ws.p + 1024 * m->f_w0z;
  v.ws = m->ws.p;
  v.ws8 = m->ws8.p;
  v.wsc_inv = (const float*)m->wsc.p;
  v.ws_frags = m->ws_frags;
  v.b0eff = (const float*)m->b0eff.p;
  v.c = (const float*)m->c.p;
  v.bc = (const float*)m->bc.p;
  v.c0 = m->c0;
  return v;
}

// Rebuild every derived operand from the FP32 master parameters.
int pack(mrdino_model* m) {
  const mrdino_dims& d = m->dims;
  const int W = d.width;
  const float* P = (const float*)m->master.p;
  hipStream_t st = m->st;
  for (int L = 0; L <= d.depth; ++L) {
    const int in = (L == 0) ? d.r_m + d.d_z : W;
    const int rows = (L == d.depth) ? d.r_u : W;
    const float* w = P + m->off_w[L];
    char* wsb = (char*)m->ws.p;
    if (L == 0) {
      saa_launch::mlp_pack_fwd(wsb + 1024 * m->f_wp[0], w, W, m->kin, W, d.r_m, in, 1, st);
      saa_launch::mlp_transpose((float*)m->wtn[0].p, w, W, d.r_m, in, st);   // r_m x W
      saa_launch::mlp_transpose((float*)m->w0zT.p, w + d.r_m, W, d.d_z, in, st);   // d_z x W (control columns)
    } else {
      saa_launch::mlp_pack_fwd(wsb + 1024 * m->f_wp[L], w, W, W, rows, W, W, 0, st);
      saa_launch::mlp_pack_bwd(wsb + 1024 * m->f_wt[L], w, W, W, rows, W, W, 0, st);
      saa_launch::mlp_transpose((float*)m->wtn[L].p, w, rows, W, W, st);     // W x rows
    }
    saa_launch::mlp_pad((float*)m->bias[L].p, P + m->off_b[L], rows, W, st);
  }
  saa_launch::mlp_add_pad((float*)m->bc.p, (const float*)m->bias[d.depth].p, (const float*)m->c.p, d.r_u, W, st);
  saa_launch::mlp_pack_bwd((char*)m->ws.p + 1024 * m->f_w0z, P + m->off_w[0], 16 * saa_launch::mlp_nzt(W), W, W,
                           d.d_z, d.r_m + d.d_z, d.r_m, st);
  // FP8 copy: operands in stream order wp[0..depth], wt[depth..1], w0z
  int64_t off[2 * MLP_MAX_DEPTH + 3];
  int n = 0;
  for (int L = 0; L <= d.depth; ++L) off[n++] = m->f_wp[L];
  for (int L = d.depth; L >= 1; --L) off[n++] = m->f_wt[L];
  off[n++] = m->f_w0z;
  off[n] = m->ws_frags;
  saa_launch::mlp_pack_fp8(m->ws.p, off, n, W, (float*)m->wsc.p, m->ws8.p, m->ws_frags, st);
  return check_hip(hipGetLastError());
}

}  // namespace saa_model

using namespace saa_model;

mrdino_model::~mrdino_model() { saa_model_free_train(this); }

extern "C" {

int mrdino_num_params(const mrdino_dims* d, int64_t* n) {
  if (!d || !n || d->width < 1 || d->depth < 1 || d->depth > MLP_MAX_DEPTH || d->r_m < 1 || d->d_z < 1 ||
      d->r_u < 1)
    return SAA_E_INVALID;
  *n = param_count(*d);
  return SAA_OK;
}

int mrdino_create(const mrdino_dims* d, void* hip_stream, mrdino_model** out) {
  if (!d || !out) return SAA_E_INVALID;
  *out = nullptr;
  if (!dims_supported(*d)) return SAA_E_INVALID;
  mrdino_model* m = new (std::nothrow) mrdino_model();
  if (!m) return SAA_E_OOM;
  static std::atomic<uint64_t> next_serial{1};
  m->serial = next_serial.fetch_add(1);
  m->dims = *d;
  m->st = (hipStream_t)hip_stream;
  m->kin = saa_launch::mlp_kin(d->width);   // columns of the BF16 layer-0 operand (r_m zero padded)
  m->n_params = param_count(*d);
  int64_t off = 0;
  int in = d->r_m + d->d_z;
  for (int L = 0; L <= d->depth; ++L) {
    const int rows = (L == d->depth) ? d->r_u : d->width;
    m->off_w[L] = off;
    off += (int64_t)rows * in;
    m->off_b[L] = off;
    off += rows;
    in = rows;
  }
  const int W = d->width;
  int rc = m->master.alloc_zero(sizeof(float) * m->n_params, m->st);
  // weight stream: wp[0..depth], wt[depth..1], w0z (the kernel's reading order)
  int64_t nf = 0;
  for (int L = 0; L <= d->depth; ++L) {
    m->f_wp[L] = nf;
    nf += (int64_t)(W / 16) * (((L == 0) ? m->kin : W) / 32);
  }
  for (int L = d->depth; L >= 1; --L) {
    m->f_wt[L] = nf;
    nf += (int64_t)(W / 16) * (W / 32);
  }
  m->f_w0z = nf;
  nf += saa_launch::mlp_nzt(W) * (W / 32);
  m->ws_frags = nf;
  if (!rc) rc = m->ws.alloc_zero(1024 * (size_t)nf, m->st);
  if (!rc) rc = m->ws8.alloc_zero(512 * (size_t)nf, m->st);
  if (!rc) rc = m->wsc.alloc_zero(sizeof(float) * (2 * MLP_MAX_DEPTH + 2), m->st);
  for (int L = 0; L <= d->depth && !rc; ++L) {
    rc = m->bias[L].alloc_zero(sizeof(float) * W, m->st);
    if (!rc) rc = m->wtn[L].alloc_zero(sizeof(float) * (size_t)W * (L == 0 ? d->r_m : W), m->st);
  }
  if (!rc) rc = m->b0eff.alloc_zero(sizeof(float) * W, m->st);
  if (!rc) rc = m->w0zT.alloc_zero(sizeof(float) * (size_t)d->d_z * W, m->st);
  if (!rc) rc = m->c.alloc_zero(sizeof(float) * W, m->st);
  if (!rc) rc = m->bc.alloc_zero(sizeof(float) * W, m->st);
  if (!rc) rc = m->zdev.alloc_zero(sizeof(double) * 64, m->st);
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  if (rc) {
    delete m;
    return rc;
  }
  *out = m;
  return SAA_OK;
}

void mrdino_free(mrdino_model* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->st);
  delete m;
}

int mrdino_set_params(mrdino_model* m, const float* params, int64_t n) {
  if (!m || !params || n != m->n_params) return SAA_E_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return SAA_E_INVALID;
  int rc = check_hip(hipMemcpyAsync(m->master.p, params, sizeof(float) * n, hipMemcpyHostToDevice, m->st));
  if (!rc) rc = pack(m);
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  return rc;
}

int mrdino_get_params(const mrdino_model* m, float* params, int64_t n) {
  if (!m || !params || n != m->n_params) return SAA_E_INVALID;
  int rc = check_hip(hipMemcpyAsync(params, m->master.p, sizeof(float) * n, hipMemcpyDeviceToHost, m->st));
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  return rc;
}

int mrdino_set_qoi(mrdino_model* m, const double* c, double c0) {
  if (!m || !c || !std::isfinite(c0)) return SAA_E_INVALID;
  const int W = m->dims.width;
  std::vector<float> buf(W, 0.0f);
  for (int i = 0; i < m->dims.r_u; ++i) {
    if (!std::isfinite(c[i])) return SAA_E_INVALID;
    buf[i] = (float)c[i];
  }
  m->c0 = c0;
  m->c_host.assign(c, c + m->dims.r_u);
  ++m->version;
  int rc = check_hip(hipMemcpyAsync(m->c.p, buf.data(), sizeof(float) * W, hipMemcpyHostToDevice, m->st));
  if (!rc) {
    saa_launch::mlp_add_pad((float*)m->bc.p, (const float*)m->bias[m->dims.depth].p, (const float*)m->c.p,
                            m->dims.r_u, W, m->st);
    rc = check_hip(hipGetLastError());
  }
  if (!rc) rc = check_hip(hipStreamSynchronize(m->st));
  return rc;
}

}  // extern "C"

// Model file: "SAADINO1", uint32 version, int32 r_m d_z r_u width depth,
// int64 n_params, float64 c0, float64 c[r_u], float32 params[n_params];
// version 2 continues with int32 has_train and, if 1, the optimiser state:
// int64 Adam step, int64 completed epochs, uint64 minibatch-stream state,
// float32 m[n_params], float32 v[n_params]; then the 64-bit FNV-1a hash of
// everything before it.  Native byte order.  Version 1 files (no optimiser
// state) still load.
namespace {
constexpr char kMagic[8] = {'S', 'A', 'A', 'D', 'I', 'N', 'O', '1'};

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 0x100000001b3ull;
  return h;
}

template <typename T>
void append(std::vector<unsigned char>& b, const T* v, size_t n) {
  const unsigned char* p = (const unsigned char*)v;
  b.insert(b.end(), p, p + sizeof(T) * n);
}

template <typename T>
bool take(const std::vector<unsigned char>& b, size_t& off, T* v, size_t n) {
  if (off + sizeof(T) * n > b.size()) return false;
  std::memcpy(v, b.data() + off, sizeof(T) * n);
  off += sizeof(T) * n;
  return true;
}
}  // namespace

extern "C" {

int mrdino_get_dims(const mrdino_model* m, mrdino_dims* d) {
  if (!m || !d) return SAA_E_INVALID;
  *d = m->dims;
  return SAA_OK;
}

int mrdino_save(const mrdino_model* m, const char* path) {
  if (!m || !path) return SAA_E_INVALID;
  std::vector<float> params(m->n_params);
  int rc = mrdino_get_params(m, params.data(), m->n_params);
  if (rc) return rc;
  std::vector<double> c(m->c_host);
  c.resize(m->dims.r_u, 0.0);
  TrainCheckpoint ck;
  if ((rc = saa_model_get_train_state(m, ck))) return rc;
  const uint32_t version = 2;
  const int32_t dims[5] = {m->dims.r_m, m->dims.d_z, m->dims.r_u, m->dims.width, m->dims.depth};
  std::vector<unsigned char> b;
  append(b, kMagic, 8);
  append(b, &version, 1);
  append(b, dims, 5);
  append(b, &m->n_params, 1);
  append(b, &m->c0, 1);
  append(b, c.data(), c.size());
  append(b, params.data(), params.size());
  const int32_t has_train = ck.present ? 1 : 0;
  append(b, &has_train, 1);
  if (ck.present) {
    append(b, &ck.step, 1);
    append(b, &ck.epoch, 1);
    append(b, &ck.rng, 1);
    append(b, ck.m.data(), ck.m.size());
    append(b, ck.v.data(), ck.v.size());
  }
  const uint64_t h = fnv1a(b.data(), b.size());
  append(b, &h, 1);
  FILE* f = std::fopen(path, "wb");
  if (!f) return SAA_E_IO;
  const bool ok = std::fwrite(b.data(), 1, b.size(), f) == b.size();
  return (std::fclose(f) == 0 && ok) ? SAA_OK : SAA_E_IO;
}

int mrdino_load(const char* path, void* hip_stream, mrdino_model** out) {
  if (!path || !out) return SAA_E_INVALID;
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return SAA_E_IO;
  std::vector<unsigned char> b;
  unsigned char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) b.insert(b.end(), chunk, chunk + got);
  std::fclose(f);
  // the whole file is validated before any device work
  if (b.size() < 8 + sizeof(uint64_t)) return SAA_E_IO;
  uint64_t h;
  std::memcpy(&h, b.data() + b.size() - sizeof(h), sizeof(h));
  if (std::memcmp(b.data(), kMagic, 8) != 0 || fnv1a(b.data(), b.size() - sizeof(h)) != h) return SAA_E_IO;
  size_t off = 8;
  uint32_t version = 0;
  int32_t dims[5];
  int64_t n = 0;
  double c0 = 0.0;
  if (!take(b, off, &version, 1) || (version != 1 && version != 2) || !take(b, off, dims, 5) ||
      !take(b, off, &n, 1) || !take(b, off, &c0, 1))
    return SAA_E_IO;
  const mrdino_dims d{dims[0], dims[1], dims[2], dims[3], dims[4]};
  if (!dims_supported(d) || n != param_count(d)) return SAA_E_IO;
  std::vector<double> c(d.r_u);
  std::vector<float> params(n);
  if (!take(b, off, c.data(), c.size()) || !take(b, off, params.data(), params.size())) return SAA_E_IO;
  TrainCheckpoint ck;
  if (version == 2) {
    int32_t has_train = 0;
    if (!take(b, off, &has_train, 1) || (has_train != 0 && has_train != 1)) return SAA_E_IO;
    if (has_train) {
      ck.present = true;
      ck.m.resize(n);
      ck.v.resize(n);
      if (!take(b, off, &ck.step, 1) || !take(b, off, &ck.epoch, 1) || !take(b, off, &ck.rng, 1) ||
          !take(b, off, ck.m.data(), ck.m.size()) || !take(b, off, ck.v.data(), ck.v.size()) || ck.step < 0 ||
          ck.epoch < 0)
        return SAA_E_IO;
    }
  }
  if (off + sizeof(h) != b.size()) return SAA_E_IO;
  mrdino_model* m = nullptr;
  int rc = mrdino_create(&d, hip_stream, &m);
  if (!rc) rc = mrdino_set_params(m, params.data(), n);
  if (!rc) rc = mrdino_set_qoi(m, c.data(), c0);
  if (!rc) rc = saa_model_set_train_state(m, ck);
  if (rc) {
    mrdino_free(m);
    return rc;
  }
  *out = m;
  return SAA_OK;
}

}  // extern "C"

// Per-sample q and dq/dz of the surrogate for the samples installed in ctx, on
// the context's stream.  z_dev: device, d_Z.  prec: SAA_FP32, SAA_BF16 or SAA_FP8.
int saa_model_eval(mrdino_model* m, saa_ctx* c, const double* z_dev, int prec, double* q, double* g) {
  const mrdino_dims& d = m->dims;
  if (d.d_z != c->dz || d.r_m > c->n_kl) return SAA_E_MODEL;
  if (prec != SAA_FP32 && prec != SAA_BF16 && prec != SAA_FP8) return SAA_E_INVALID;
  saa_launch::mlp_b0eff((float*)m->b0eff.p, (const float*)m->w0zT.p, (const float*)m->master.p + m->off_b[0], z_dev,
                        d.width, d.d_z, c->st);
  const MlpDev v = view(m);
  if (prec != SAA_FP32 && c->enc_rm != enc_key(d.r_m, m->kin)) {   // encode the installed samples once
    const size_t bytes = sizeof(uint16_t) * (size_t)m->kin * (size_t)c->N_max;
    int rc = c->enc.bytes >= bytes ? SAA_OK : c->enc.alloc(bytes);
    if (rc) return rc;
    saa_launch::mlp_encode((const double*)c->xi.p, (int)c->n_kl, (const int*)c->order.p, d.r_m, m->kin, c->N,
                           c->enc.p, c->st);
    if ((rc = check_hip(hipGetLastError()))) return rc;
    c->enc_rm = enc_key(d.r_m, m->kin);
  }
  const int rc = saa_launch::mlp_eval(v, prec == SAA_FP32 ? 0 : prec == SAA_BF16 ? 1 : 2, (const double*)c->xi.p,
                                      (int)c->n_kl, (const int*)c->order.p, c->enc.p, c->N, q, g, 0, c->st);
  if (rc) return SAA_E_DEVICE;
  return check_hip(hipGetLastError());
}

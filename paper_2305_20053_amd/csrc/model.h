// Internal definition of the MR-DINO model object.
#pragma once
#include <vector>

#include "ctx.h"
#include "mlp.h"

struct mrdino_model {
  mrdino_dims dims{};
  hipStream_t st = nullptr;
  int kin = 0;                              // columns of the BF16 layer-0 operand
  int64_t n_params = 0;
  int64_t off_w[MLP_MAX_DEPTH + 1] = {};   // offsets of W_L, b_L in the packed parameters
  int64_t off_b[MLP_MAX_DEPTH + 1] = {};
  saa_rt::DevBuf master;                    // FP32 parameters
  saa_rt::DevBuf ws;                        // BF16 MFMA operands (weight stream)
  saa_rt::DevBuf ws8, wsc;                  // FP8 copy and its per-operand 1 / scale
  int64_t ws_frags = 0;                     // stream length in 1 KB fragments
  int64_t f_wp[MLP_MAX_DEPTH + 1] = {};     // fragment offsets of the operands in the stream
  int64_t f_wt[MLP_MAX_DEPTH + 1] = {};
  int64_t f_w0z = 0;
  saa_rt::DevBuf bias[MLP_MAX_DEPTH + 1];   // FP32 biases padded to width
  saa_rt::DevBuf wtn[MLP_MAX_DEPTH + 1];    // FP32 transposed weights (reference kernel)
  saa_rt::DevBuf b0eff, c, zdev;
  saa_rt::DevBuf w0zT;                      // control columns of W_0, transposed (d_z x width), FP32
  saa_rt::DevBuf bc;                        // output bias + c (padded), for the BF16 kernel
  double c0 = 0.0;
  std::vector<double> c_host;               // c as given to mrdino_set_qoi (zeros until set)
  void* train = nullptr;                    // training workspace and Adam state (train.cpp)
  uint64_t serial = 0;                      // unique per model object (keys captured graphs)
  uint64_t version = 0;                     // bumped whenever c, c0 change: a captured graph holds c0
                                            // by value, so it keys graphs too (weights and c are read
                                            // from device buffers whose addresses never change)
  ~mrdino_model();
};

// Releases the training state of a model (train.cpp).
void saa_model_free_train(mrdino_model* m);

// Optimiser state of a model for checkpoints (train.cpp): Adam moments, step,
// completed epochs and the minibatch-order stream.  present = false: the
// model has not been trained.
struct TrainCheckpoint {
  bool present = false;
  int64_t step = 0, epoch = 0;
  uint64_t rng = 0;
  std::vector<float> m, v;
};
int saa_model_get_train_state(const mrdino_model* m, TrainCheckpoint& ck);
int saa_model_set_train_state(mrdino_model* m, const TrainCheckpoint& ck);

namespace saa_model {
int pack(mrdino_model* m);
MlpDev view(const mrdino_model* m);
}  // namespace saa_model

// Key of the BF16 encoding a context holds: r_m leading coordinates padded to kin.
inline int enc_key(int r_m, int kin) { return r_m * 4096 + kin; }

// Surrogate q and dq/dz for the installed samples (device outputs, ctx stream).
int saa_model_eval(mrdino_model* m, saa_ctx* c, const double* z_dev, int prec, double* q, double* g);

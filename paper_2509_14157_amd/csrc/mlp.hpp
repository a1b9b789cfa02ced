// Learned initial guess: a small MLP over per-element features of T3.
//
// Network: kFeat -> 256 -> 256 -> 2, SiLU after the two hidden layers.
// Outputs per T3 element: y0, the correction to the MP-style guess in units
// of its RMS (t3 = x + sx * y0), and y1, the shift of the element's Jacobi
// denominator (Eh).  Training is FP32 on the device (MFMA GEMMs, Adam);
// inference runs the GEMMs with single-BF16 operands and FP32 accumulation.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace fno {

class Mlp {
 public:
  static constexpr int F = mlp::kFeat, H = 256, O = 2;
  explicit Mlp(int device);
  ~Mlp();
  Mlp(const Mlp&) = delete;
  Mlp& operator=(const Mlp&) = delete;

  int device;
  hipStream_t stream = nullptr;
  std::string err;

  // parameters, flat: W1[F][H], b1[H], W2[H][H], b2[H], W3[H][O], b3[O] (row-major)
  static int64_t num_params() { return (int64_t)F * H + H + (int64_t)H * H + H + (int64_t)H * O + O; }
  void init(uint64_t seed);
  void get_params(float* host) const;
  void set_params(const float* host);
  void save(const std::string& path) const;
  void load(const std::string& path);

  // training set on the device (appended by the feature extraction of a context)
  void reserve(int64_t ns, float** X, float** T);  // rows X[ns][F] and T[ns][2] for the caller to fill
  void commit(int64_t ns);
  int64_t samples() const { return n_; }
  void read_samples(float* X, float* T, int64_t n) const;  // first n rows, host
  void clear_samples() { n_ = 0; }
  // minibatch Adam over the set; returns the mean loss of the last 100 steps
  double train(int steps, int batch, double lr, uint64_t seed);
  // loss and gradient of one batch (device pointers), gradient into g_
  double loss_grad(const float* X, const float* T, int64_t B);
  const float* grad() const { return g_; }
  float out_weight[O] = {1.0f, 1.0f};

  // BF16 inference: Y[n][O] = net(X[n][F]) (device pointers), in chunks
  void predict_bf16(const float* X, int64_t n, float* Y, hipStream_t s);

 private:
  float *p_ = nullptr, *g_ = nullptr, *m_ = nullptr, *v_ = nullptr, *w_ = nullptr;
  float* X_ = nullptr;  // dataset features
  float* T_ = nullptr;  // dataset targets
  int64_t n_ = 0, cap_ = 0, pending_ = 0;
  int step_ = 0;
  // work buffers for a batch of B rows
  int64_t wb_ = 0;
  float *Z1_ = nullptr, *A1_ = nullptr, *Z2_ = nullptr, *A2_ = nullptr, *Y_ = nullptr, *dY_ = nullptr,
        *dA_ = nullptr, *dZ_ = nullptr, *part_ = nullptr, *Xb_ = nullptr, *Tb_ = nullptr;
  // BF16 inference buffers
  int64_t ib_ = 0;
  void *wh_ = nullptr, *wl_ = nullptr, *ah_ = nullptr, *al_ = nullptr;
  float *iz_ = nullptr, *ia_ = nullptr;
  void* ws_ = nullptr;  // split-K partials of the GEMMs
  size_t ws_bytes_ = 0;
  void ensure_batch(int64_t B);
  void ensure_infer(int64_t B);
  void forward(const float* X, int64_t B);
  void backward(const float* X, const float* T, int64_t B);
  double read_loss(int64_t B);
  float* W1() const { return p_; }
  float* b1() const { return p_ + F * H; }
  float* W2() const { return b1() + H; }
  float* b2() const { return W2() + H * H; }
  float* W3() const { return b2() + H; }
  float* b3() const { return W3() + H * O; }
};

}  // namespace fno

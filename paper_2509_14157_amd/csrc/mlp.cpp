// Learned initial guess: MLP training and inference on the device.
#include "mlp.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace fno {

namespace {
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

float* dalloc(int64_t n) {
  float* p = nullptr;
  FNO_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(float)));
  FNO_HIP(hipMemset(p, 0, (size_t)std::max<int64_t>(n, 1) * sizeof(float)));
  return p;
}

void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// C = alpha A B + beta C with the library's MFMA GEMM (FP32 or single-BF16 operands)
void gemm(Prec prec, const void* A, const void* Alo, int64_t lda, bool akf, const void* B, const void* Blo,
          int64_t ldb, bool bnf, void* C, int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha, double beta,
          void*& ws, size_t& ws_bytes, hipStream_t s) {
  GemmArgs g{};
  g.prec = prec;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.A_lo = Alo;
  g.lda = lda;
  g.a_kfast = akf;
  g.B = B;
  g.B_lo = Blo;
  g.ldb = ldb;
  g.b_nfast = bnf;
  g.C = C;
  g.ldc = ldc;
  g.alpha = alpha;
  g.beta = beta;
  g.tile = -1;
  g.split = gemm_split_factor(g);
  if (g.split > 1) {
    const size_t need = gemm_split_bytes(g, g.split);
    if (need > ws_bytes) {
      FNO_HIP(hipStreamSynchronize(s));
      dfree(ws);
      FNO_HIP(hipMalloc(&ws, need));
      ws_bytes = need;
    }
    g.ws = ws;
  }
  launch_gemm(g, s);
}
}  // namespace

Mlp::Mlp(int dev) : device(dev) {
  FNO_HIP(hipSetDevice(device));
  FNO_HIP(hipStreamCreate(&stream));
  const int64_t np = num_params();
  p_ = dalloc(np);
  g_ = dalloc(np);
  m_ = dalloc(np);
  v_ = dalloc(np);
  w_ = dalloc(O);
  init(1);
}

Mlp::~Mlp() {
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (void* q : {(void*)p_, (void*)g_, (void*)m_, (void*)v_, (void*)w_, (void*)X_, (void*)T_, (void*)Z1_, (void*)A1_,
                  (void*)Z2_, (void*)A2_, (void*)Y_, (void*)dY_, (void*)dA_, (void*)dZ_, (void*)part_, (void*)Xb_,
                  (void*)Tb_, wh_, wl_, ah_, al_, (void*)iz_, (void*)ia_, ws_})
    if (q) (void)hipFree(q);
  if (stream) (void)hipStreamDestroy(stream);
}

void Mlp::init(uint64_t seed) {
  std::vector<float> h(num_params(), 0.0f);
  uint64_t s = seed;
  auto fill = [&](float* w, int fin, int fout, float gain) {
    const float a = gain * std::sqrt(6.0f / (float)(fin + fout));
    for (int64_t i = 0; i < (int64_t)fin * fout; ++i) {
      const double u = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0);
      w[i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  float* base = h.data();
  fill(base, F, H, 1.0f);
  fill(base + F * H + H, H, H, 1.0f);
  // small output layer: an untrained network leaves the MP-style guess unchanged
  fill(base + F * H + H + H * H + H, H, O, 0.1f);
  set_params(h.data());
  FNO_HIP(hipMemset(m_, 0, num_params() * sizeof(float)));
  FNO_HIP(hipMemset(v_, 0, num_params() * sizeof(float)));
  step_ = 0;
}

void Mlp::get_params(float* host) const {
  FNO_HIP(hipStreamSynchronize(stream));
  FNO_HIP(hipMemcpy(host, p_, num_params() * sizeof(float), hipMemcpyDeviceToHost));
}

void Mlp::set_params(const float* host) {
  FNO_HIP(hipStreamSynchronize(stream));
  FNO_HIP(hipMemcpy(p_, host, num_params() * sizeof(float), hipMemcpyHostToDevice));
}

void Mlp::save(const std::string& path) const {
  std::vector<float> h(num_params());
  get_params(h.data());
  FILE* f = std::fopen(path.c_str(), "wb");
  FNO_REQUIRE(f != nullptr, kEINVAL, "cannot open " + path + " for writing");
  const char magic[8] = {'F', 'N', 'O', 'M', 'L', 'P', '0', '1'};
  const int32_t dims[3] = {F, H, O};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, 4, 3, f) == 3 &&
            std::fwrite(h.data(), 4, h.size(), f) == h.size();
  std::fclose(f);
  FNO_REQUIRE(ok, kEINVAL, "short write to " + path);
}

void Mlp::load(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  FNO_REQUIRE(f != nullptr, kEINVAL, "cannot open " + path);
  char magic[8];
  int32_t dims[3];
  std::vector<float> h(num_params());
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "FNOMLP01", 8) == 0 &&
            std::fread(dims, 4, 3, f) == 3 && dims[0] == F && dims[1] == H && dims[2] == O &&
            std::fread(h.data(), 4, h.size(), f) == h.size();
  std::fclose(f);
  FNO_REQUIRE(ok, kEINVAL, "not a weights file of this network: " + path);
  for (float x : h) FNO_REQUIRE(std::isfinite(x), kENONFINITE, "non-finite weight in " + path);
  set_params(h.data());
}

void Mlp::reserve(int64_t ns, float** Xo, float** To) {
  if (n_ + ns > cap_) {
    const int64_t cap = std::max<int64_t>(2 * cap_, n_ + ns);
    float* X = dalloc(cap * F);
    float* T = dalloc(cap * 2);
    if (n_) {
      FNO_HIP(hipMemcpy(X, X_, n_ * F * sizeof(float), hipMemcpyDeviceToDevice));
      FNO_HIP(hipMemcpy(T, T_, n_ * 2 * sizeof(float), hipMemcpyDeviceToDevice));
    }
    dfree((void*&)X_);
    dfree((void*&)T_);
    X_ = X;
    T_ = T;
    cap_ = cap;
  }
  pending_ = ns;
  *Xo = X_ + n_ * F;
  *To = T_ + n_ * 2;
}

void Mlp::read_samples(float* X, float* T, int64_t n) const {
  FNO_REQUIRE(n >= 0 && n <= n_, kEINVAL, "more rows than collected samples");
  FNO_HIP(hipDeviceSynchronize());
  FNO_HIP(hipMemcpy(X, X_, (size_t)n * F * sizeof(float), hipMemcpyDeviceToHost));
  FNO_HIP(hipMemcpy(T, T_, (size_t)n * 2 * sizeof(float), hipMemcpyDeviceToHost));
}

void Mlp::commit(int64_t ns) {
  FNO_REQUIRE(ns <= pending_, kEINVAL, "commit beyond the reserved rows");
  n_ += ns;
  pending_ = 0;
}

void Mlp::ensure_batch(int64_t B) {
  if (B <= wb_) return;
  FNO_HIP(hipStreamSynchronize(stream));
  for (float** q : {&Z1_, &A1_, &Z2_, &A2_, &dA_, &dZ_}) {
    dfree((void*&)*q);
    *q = dalloc(B * H);
  }
  for (float** q : {&Y_, &dY_, &Tb_}) {
    dfree((void*&)*q);
    *q = dalloc(B * O);
  }
  dfree((void*&)Xb_);
  Xb_ = dalloc(B * F);
  dfree((void*&)part_);
  part_ = dalloc(1024);
  wb_ = B;
}

void Mlp::forward(const float* X, int64_t B) {
  gemm(Prec::FP32, X, nullptr, F, true, W1(), nullptr, H, true, Z1_, H, B, H, F, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::bias_act(Z1_, b1(), A1_, B, H, true, stream);
  gemm(Prec::FP32, A1_, nullptr, H, true, W2(), nullptr, H, true, Z2_, H, B, H, H, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::bias_act(Z2_, b2(), A2_, B, H, true, stream);
  gemm(Prec::FP32, A2_, nullptr, H, true, W3(), nullptr, O, true, Y_, O, B, O, H, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::bias_act(Y_, b3(), Y_, B, O, false, stream);
}

// forward, weighted MSE and backward of one batch; the gradient lands in g_,
// the per-block loss partials in part_ (nothing is read back)
void Mlp::backward(const float* X, const float* T, int64_t B) {
  ensure_batch(B);
  FNO_HIP(hipMemcpyAsync(w_, out_weight, O * sizeof(float), hipMemcpyHostToDevice, stream));
  forward(X, B);
  mlp::mse(Y_, T, w_, dY_, part_, B, O, stream);
  float* gW1 = g_;
  float* gb1 = g_ + F * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H * O;
  // output layer: dW3 = A2^T dY, db3 = sum dY, dA2 = dY W3^T
  gemm(Prec::FP32, A2_, nullptr, H, false, dY_, nullptr, O, true, gW3, O, H, O, B, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::colsum(dY_, gb3, B, O, stream);
  gemm(Prec::FP32, dY_, nullptr, O, true, W3(), nullptr, O, false, dA_, H, B, H, O, 1.0, 0.0, ws_, ws_bytes_, stream);
  // second hidden layer
  mlp::act_grad(Z2_, dA_, dZ_, B * H, stream);
  gemm(Prec::FP32, A1_, nullptr, H, false, dZ_, nullptr, H, true, gW2, H, H, H, B, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::colsum(dZ_, gb2, B, H, stream);
  gemm(Prec::FP32, dZ_, nullptr, H, true, W2(), nullptr, H, false, dA_, H, B, H, H, 1.0, 0.0, ws_, ws_bytes_, stream);
  // first hidden layer
  mlp::act_grad(Z1_, dA_, dZ_, B * H, stream);
  gemm(Prec::FP32, X, nullptr, F, false, dZ_, nullptr, H, true, gW1, H, F, H, B, 1.0, 0.0, ws_, ws_bytes_, stream);
  mlp::colsum(dZ_, gb1, B, H, stream);
}

double Mlp::read_loss(int64_t B) {
  const int nb = mlp::mse_blocks(B * O);
  std::vector<float> part(nb);
  FNO_HIP(hipMemcpyAsync(part.data(), part_, nb * sizeof(float), hipMemcpyDeviceToHost, stream));
  FNO_HIP(hipStreamSynchronize(stream));
  double l = 0;
  for (float x : part) l += x;
  return l;
}

double Mlp::loss_grad(const float* X, const float* T, int64_t B) {
  backward(X, T, B);
  return read_loss(B);
}

double Mlp::train(int steps, int batch, double lr, uint64_t seed) {
  FNO_REQUIRE(n_ > 0, kESTATE, "no training samples");
  FNO_REQUIRE(steps >= 1 && batch >= 1, kEINVAL, "bad training options");
  ensure_batch(batch);
  double tail = 0;
  int ntail = 0;
  for (int s = 0; s < steps; ++s) {
    mlp::gather(X_, T_, Xb_, Tb_, n_, batch, seed * 1000003ull + (uint64_t)s, stream);
    backward(Xb_, Tb_, batch);
    if (s >= steps - 20) {
      tail += read_loss(batch);
      ++ntail;
    }
    ++step_;
    mlp::adam(p_, g_, m_, v_, num_params(), (float)lr, 0.9f, 0.999f, 1e-8f, step_, stream);
  }
  FNO_HIP(hipStreamSynchronize(stream));
  return ntail ? tail / ntail : 0.0;
}

void Mlp::ensure_infer(int64_t B) {
  if (B <= ib_ && wh_) return;
  FNO_HIP(hipStreamSynchronize(stream));
  for (void** q : {&ah_, &al_}) {
    dfree(*q);
    FNO_HIP(hipMalloc(q, (size_t)B * H * 2));
  }
  dfree((void*&)iz_);
  dfree((void*&)ia_);
  iz_ = dalloc(B * H);
  ia_ = dalloc(B * H);
  if (!wh_) {
    FNO_HIP(hipMalloc(&wh_, (size_t)num_params() * 2));
    FNO_HIP(hipMalloc(&wl_, (size_t)num_params() * 2));
  }
  ib_ = B;
}

void Mlp::predict_bf16(const float* X, int64_t n, float* Y, hipStream_t s) {
  const int64_t chunk = 1 << 20;
  ensure_infer(std::min<int64_t>(n, chunk));
  // the caller's stream orders the inputs; weights are read on it as well
  FNO_HIP(hipStreamSynchronize(stream));
    mlp::to_bf16(p_, wh_, wl_, num_params(), s);
  const int64_t oW1 = 0, oW2 = (int64_t)F * H + H, oW3 = oW2 + (int64_t)H * H + H;
  auto wptr = [&](void* base, int64_t off) { return (void*)((char*)base + off * 2); };
  for (int64_t r0 = 0; r0 < n; r0 += chunk) {
    const int64_t B = std::min(chunk, n - r0);
    mlp::to_bf16(X + r0 * F, ah_, al_, B * F, s);
    gemm(Prec::BF16X3, ah_, al_, F, true, wptr(wh_, oW1), wptr(wl_, oW1), H, true, iz_, H, B, H, F, 1.0, 0.0, ws_,
         ws_bytes_, s);
    mlp::bias_act(iz_, b1(), ia_, B, H, true, s);
    mlp::to_bf16(ia_, ah_, al_, B * H, s);
    gemm(Prec::BF16X3, ah_, al_, H, true, wptr(wh_, oW2), wptr(wl_, oW2), H, true, iz_, H, B, H, H, 1.0, 0.0, ws_,
         ws_bytes_, s);
    mlp::bias_act(iz_, b2(), ia_, B, H, true, s);
    mlp::to_bf16(ia_, ah_, al_, B * H, s);
    float* y = Y + r0 * O;
    gemm(Prec::BF16X3, ah_, al_, H, true, wptr(wh_, oW3), wptr(wl_, oW3), O, true, y, O, B, O, H, 1.0, 0.0, ws_,
         ws_bytes_, s);
    mlp::bias_act(y, b3(), y, B, O, false, s);
  }
}

}  // namespace fno

// Context-free entry point of the fused triples residual (triples.hpp) on
// caller device buffers: the same kernels as the context's residual sweep,
// with their working buffers (T3v, W3_vvvv^T, the products Y, the ring
// operand, the padded F3_vv, the occupied-only operator) carved out of one
// scratch block.
#include <cstring>
#include <mutex>
#include <string>

#include "triples_dev.hpp"

#include "kernels.hpp"

namespace fno {
namespace {

constexpr int kDevMaxN = 64;  // occupied and virtual sizes these entry points take

constexpr int kDec2 = kDevMaxN * (kDevMaxN - 1) / 2;
constexpr int kDec3 = kDevMaxN * (kDevMaxN - 1) * (kDevMaxN - 2) / 6;

// colex decode tables of pairs and triples of indices below kDevMaxN, filled
// on the device once per device (the fused kernels read them)
static __device__ uint8_t g_dec2[2 * kDec2];
static __device__ uint8_t g_dec3[3 * kDec3];

__global__ void dec_tables_kernel(uint8_t* d2, uint8_t* d3) {
  // thread per largest element c: its pairs (b < c) and triples (a < b < c)
  // follow those of every smaller c, in colex order
  const int c = threadIdx.x;
  if (c >= kDevMaxN) return;
  int p = c * (c - 1) / 2;
  for (int b = 0; b < c; ++b, ++p) {
    d2[2 * p] = (uint8_t)b;
    d2[2 * p + 1] = (uint8_t)c;
  }
  int q = c * (c - 1) * (c - 2) / 6;
  for (int b = 1; b < c; ++b)
    for (int a = 0; a < b; ++a, ++q) {
      d3[3 * q] = (uint8_t)a;
      d3[3 * q + 1] = (uint8_t)b;
      d3[3 * q + 2] = (uint8_t)c;
    }
}

struct DevState {
  bool ready = false;
  IndexTables tb{};
};
std::mutex g_mu;
DevState g_dev[kDevMaxDevices];

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

thread_local std::string g_dev_err;

IndexTables dev_tables(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  DevState& st = g_dev[device];
  if (!st.ready) {
    void *d2 = nullptr, *d3 = nullptr;
    FNO_HIP(hipGetSymbolAddress(&d2, HIP_SYMBOL(g_dec2)));
    FNO_HIP(hipGetSymbolAddress(&d3, HIP_SYMBOL(g_dec3)));
    dec_tables_kernel<<<1, kDevMaxN, 0, nullptr>>>((uint8_t*)d2, (uint8_t*)d3);
    FNO_HIP(hipGetLastError());
    FNO_HIP(hipDeviceSynchronize());
    st.tb.dec[2] = (const uint8_t*)d2;
    st.tb.dec[3] = (const uint8_t*)d3;
    st.tb.dec_max_n[2] = kDevMaxN;
    st.tb.dec_max_n[3] = kDevMaxN;
    st.ready = true;
  }
  return st.tb;
}

Layout layout(int o, int v, Prec p) {
  const size_t es = p == Prec::FP64 ? 8 : 4;
  const size_t nt = (size_t)binom_host(o, 3);
  Layout L{};
  size_t off = 0;
  L.t3v = off;
  off += up256(es * (size_t)r3_fused_t3v_elems(o, v));
  L.wt = off;
  off += up256(es * (size_t)r3_fused_wt_elems(v));
  L.y = off;
  off += up256(es * (size_t)r3_fused_y_elems(o, v));
  L.aring = off;
  off += up256(8 * (size_t)r3_ring_operand_elems(o, v));
  L.fvvp = off;
  off += up256(8 * (size_t)r3_fvv_padded_elems(v));
  L.occ = off;
  off += up256(8 * nt * nt);
  L.total = off;
  return L;
}

void run_pass(const IndexTables& tb, int o, int v, Prec prec, const Inputs& in, double* R3, unsigned char* base,
              hipStream_t s) {
  const Layout L = layout(o, v, prec);
  const int nt = (int)binom_host(o, 3), nv3 = (int)binom_host(v, 3);
  void* t3v = base + L.t3v;
  void* wt = base + L.wt;
  void* y = base + L.y;
  double* aring = (double*)(base + L.aring);
  double* fvvp = (double*)(base + L.fvvp);
  double* occ = (double*)(base + L.occ);
  launch_r3_operands(tb, o, v, in.T3, in.Wvvvv, t3v, wt, prec, s);
  launch_r3_ring_operand(in.Wovvo, in.Fvv, o, v, aring, fvvp, s);
  launch_r3_occ_operator(tb, o, in.Woooo, in.Foo, occ, s);
  R3FusedArgs a;
  a.o = o;
  a.v = v;
  a.T3 = in.T3;
  a.T3v = t3v;
  a.WT = wt;
  a.T2 = in.T2;
  a.Wvvvv = in.Wvvvv;
  a.Fvvp = fvvp;
  a.Aring = aring;
  a.Wvvvo = in.Wvvvo;
  a.Wovoo = in.Wovoo;
  a.Y = y;
  a.ldy = r3_fused_ldy(v);
  launch_r3_fused(tb, a, prec, s);
  launch_r3_fold(tb, o, v, y, a.ldy, prec, R3, s);
  GemmArgs g{};
  g.prec = Prec::FP64;
  g.M = nt;
  g.N = nv3;
  g.K = nt;
  g.A = occ;
  g.lda = nt;
  g.a_kfast = true;
  g.B = in.T3;
  g.ldb = nv3;
  g.b_nfast = true;
  g.C = R3;
  g.ldc = nv3;
  g.alpha = 1.0;
  g.beta = 1.0;
  g.tile = -1;
  g.split = 1;
  launch_gemm(g, s);
}

Prec check_args(int device, int o, int v, fno_prec prec, const Inputs& in, const double* R3) {
  int ndev = 0;
  FNO_HIP(hipGetDeviceCount(&ndev));
  FNO_REQUIRE(device >= 0 && device < ndev && device < kDevMaxDevices, kEDEVICE, "no such HIP device");
  FNO_REQUIRE(o >= 3 && o <= kDevMaxN && v >= 3 && v <= kDevMaxN, kEINVAL,
              "the fused triples residual takes 3 <= nocc <= 64 and 3 <= nvir <= 64");
  FNO_REQUIRE(prec == FNO_FP64 || prec == FNO_FP32 || prec == FNO_BF16X3, kEINVAL,
              "the fused triples residual runs FP64, FP32 or split-BF16 products");
  FNO_REQUIRE(in.T3 && in.T2 && in.Wvvvv && in.Fvv && in.Wovvo && in.Wvvvo && in.Wovoo && in.Woooo && in.Foo && R3,
              kEINVAL, "null device buffer");
  return prec == FNO_FP64 ? Prec::FP64 : (prec == FNO_FP32 ? Prec::FP32 : Prec::BF16X3);
}

}  // namespace fno

extern "C" {

const char* fno_dev_last_error(void) { return fno::g_dev_err.c_str(); }

int fno_triples_residual_dev(int hip_device, int nocc, int nvir, fno_prec prec, const double* T3, const double* T2,
                             const double* W3_vvvv, const double* F3_vv, const double* W3_ovvo,
                             const double* W3_vvvo, const double* W3_ovoo, const double* W3_oooo,
                             const double* F3_oo, double* R3, void* stream) {
  return fno::dev_guard([&]() {
    const fno::Inputs in{T3, T2, W3_vvvv, F3_vv, W3_ovvo, W3_vvvo, W3_ovoo, W3_oooo, F3_oo};
    const fno::Prec p = fno::check_args(hip_device, nocc, nvir, prec, in, R3);
    FNO_HIP(hipSetDevice(hip_device));
    const fno::IndexTables tb = fno::dev_tables(hip_device);
    const hipStream_t s = (hipStream_t)stream;
    const fno::Layout L = fno::layout(nocc, nvir, p);
    unsigned char* work = nullptr;
    FNO_HIP(hipMalloc((void**)&work, L.total));
    try {
      fno::run_pass(tb, nocc, nvir, p, in, R3, work, s);
      FNO_HIP(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(work);
      throw;
    }
    FNO_HIP(hipFree(work));
    return FNO_OK;
  });
}

}  // extern "C"

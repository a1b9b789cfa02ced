// The fused triples residual entry point that allocates nothing: its working
// buffers live in one file-scope device array of fixed size, each device's
// copy looked up once (hipGetSymbolAddress, that device current) and passed
// to the kernels as a plain pointer.
#include <mutex>

#include "triples_dev.hpp"

namespace fno {
namespace {

// 256 MiB per device, held from the first use on that device until the
// process ends: enough for the o=10, v=59 and o=12, v=48 workloads in FP64
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_scratch[kDevMaxDevices] = {};

// this device's copy of `scratch` (the device is current)
unsigned char* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    FNO_REQUIRE(rc == hipSuccess && p != nullptr, kEDEVICE,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(rc));
    g_scratch[device] = (unsigned char*)p;
  }
  return g_scratch[device];
}

}  // namespace
}  // namespace fno

extern "C" int fno_triples_residual_dev_noalloc(int hip_device, int nocc, int nvir, fno_prec prec,
                                                const double* T3, const double* T2, const double* W3_vvvv,
                                                const double* F3_vv, const double* W3_ovvo, const double* W3_vvvo,
                                                const double* W3_ovoo, const double* W3_oooo, const double* F3_oo,
                                                double* R3, void* stream) {
  return fno::dev_guard([&]() {
    const fno::Inputs in{T3, T2, W3_vvvv, F3_vv, W3_ovvo, W3_vvvo, W3_ovoo, W3_oooo, F3_oo};
    const fno::Prec p = fno::check_args(hip_device, nocc, nvir, prec, in, R3);
    const fno::Layout L = fno::layout(nocc, nvir, p);
    FNO_REQUIRE(L.total <= fno::kScratchBytes, FNO_ENOMEM,
                "nocc = " + std::to_string(nocc) + ", nvir = " + std::to_string(nvir) + " needs " +
                    std::to_string(L.total) + " bytes of working memory; the static buffer holds " +
                    std::to_string(fno::kScratchBytes) + " (use fno_triples_residual_dev)");
    FNO_HIP(hipSetDevice(hip_device));
    const fno::IndexTables tb = fno::dev_tables(hip_device);
    unsigned char* base = fno::scratch_ptr(hip_device);
    fno::run_pass(tb, nocc, nvir, p, in, R3, base, (hipStream_t)stream);
    return FNO_OK;
  });
}

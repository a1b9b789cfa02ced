// Contraction engine: packed antisymmetric tensors and einsum-like terms.
//
// A term  Out[ijkabc] += alpha * A[ijkaef] * B[bcef]  means
//   Out += alpha * P( sum_{e,f} A * B )
// where P sums over the coset representatives of the output's antisymmetry
// group modulo the antisymmetry the product already has (the usual
// P(a/bc), P(k/ij)P(a/bc), ... operators of spin-orbital coupled cluster).
// The planner turns a term into: optional expansion of each operand into a
// GEMM matrix (gathering from packed storage with signs), one MFMA GEMM, and
// an optional fold of the GEMM result into the packed output.  Summation
// letters that are antisymmetric in both operands are summed over ordered
// tuples only (times g!), output letters that are antisymmetric in an
// operand are produced as ordered tuples only.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace fno {

struct Group {
  int g = 1;       // slots in the group (all of one index space)
  int n = 0;       // index range seen through this tensor (view extent)
  int off = 0;     // view offset (g == 1 only)
  int ext = 0;     // storage extent of the index space
  int64_t count() const { return g == 1 ? n : (int64_t)binom_host(n, g); }
  int64_t storage() const { return g == 1 ? ext : (int64_t)binom_host(ext, g); }
};

struct Tensor {
  std::string name;
  std::vector<Group> groups;
  // Antisymmetry partition of the slots (slot index lists).  For packed
  // tensors it equals the storage groups; a dense tensor may declare
  // antisymmetric slot sets without packing them (e.g. <pq||rs>).
  std::vector<std::vector<int>> sym;
  double* d = nullptr;      // device data (FP64)
  int64_t base = 0;         // view origin (elements)
  int64_t elems = 0;        // storage elements of the whole buffer
  bool owner = false;
  int nslots() const {
    int s = 0;
    for (auto& g : groups) s += g.g;
    return s;
  }
  std::vector<int64_t> strides() const {
    std::vector<int64_t> st(groups.size());
    int64_t s = 1;
    for (int q = (int)groups.size() - 1; q >= 0; --q) {
      st[q] = s;
      s *= groups[q].storage();
    }
    return st;
  }
  bool full_view() const {
    if (base != 0) return false;
    for (auto& g : groups)
      if (g.off != 0 || g.n != g.ext) return false;
    return true;
  }
  int64_t view_size() const {
    int64_t s = 1;
    for (auto& g : groups) s *= g.count();
    return s;
  }
};

// Storage spec "ooo,vvv": comma-separated groups, one character per slot.
struct SpaceSizes {
  std::map<char, int> n;
};

struct GemmStats {
  std::string term;
  int64_t M = 0, N = 0, K = 0;
  double flops = 0;
};

class Engine {
 public:
  explicit Engine(int device);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  hipStream_t stream = nullptr;
  Prec prec = Prec::FP64;
  IndexTables tables{};
  int device = 0;

  // --- tensors
  // Allocate a zeroed tensor; with `external` the tensor lives in caller memory.
  Tensor* create(const std::string& name, const std::string& spec, const SpaceSizes& sz,
                 double* external = nullptr);
  static int64_t spec_size(const std::string& spec, const SpaceSizes& sz);
  Tensor* view(const std::string& name, Tensor* parent, const std::vector<std::pair<int, int>>& ranges);
  Tensor* get(const std::string& name) const;
  void set_sym(Tensor* t, const std::vector<std::vector<int>>& sym);
  bool has(const std::string& name) const { return reg_.count(name) != 0; }
  void drop(const std::string& name);
  void zero(Tensor* t);

  // --- terms
  void term(const std::string& spec, double scale = 1.0);
  void terms(const char* const* specs, int n, double scale = 1.0);

  // --- statistics (per-term algorithmic flops of the GEMMs issued)
  bool record = false;
  std::vector<GemmStats> stats;

  // --- per-kernel profiling with HIP events on `stream`
  bool profile = false;
  void prof_mark(const std::string& label, const std::string& spec, double flops, double bytes, hipEvent_t a,
                 hipEvent_t b);
  hipEvent_t event();
  std::string profile_report();  // JSON aggregate per kernel label; clears the records

  // workspace sizes (bytes) currently held
  size_t workspace_bytes() const { return ws_bytes_[0] + ws_bytes_[1] + ws_bytes_[2] + ws_bytes_[3] + ws_bytes_[4] + ws_bytes_[5]; }
  void* workspace(int slot, size_t bytes);

  // device buffers for tables
 private:
  struct Plan;
  std::map<std::string, std::unique_ptr<Tensor>> reg_;
  std::map<std::string, std::shared_ptr<Plan>> plans_;
  void* ws_[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t ws_bytes_[6] = {0, 0, 0, 0, 0, 0};
  uint32_t* d_binom_ = nullptr;
  uint8_t* d_dec_[kMaxGroup + 1] = {};
  struct ProfRec {
    std::string label, spec;
    double flops, bytes;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_;
  std::vector<hipEvent_t> evpool_;
  size_t evnext_ = 0;
  std::shared_ptr<Plan> plan(const std::string& spec);
  void execute(const Plan& p, double scale);
};

}  // namespace fno

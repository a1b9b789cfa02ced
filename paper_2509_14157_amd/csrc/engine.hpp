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

#include <algorithm>
#include <functional>
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

// A recorded sequence of launches (one instantiated hipGraph; empty when
// nothing was captured), with the kernels timed inside it.
struct Program {
  struct Item {
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Item> items;
  // kernels timed inside the graph: event-record nodes around them, read
  // after every replay
  struct Timer {
    std::string label, spec;
    double flops, bytes;
    hipEvent_t a, b;
  };
  std::vector<Timer> timers;
  // the last replay's timers have not been read yet (deferred replay)
  mutable bool pending = false;
  uint64_t epoch = 0;  // engine epoch the recording is valid for
  int prec = -1;
  bool profiled = false;
  std::string filter;
  // stream of the last replay: a replay may still run when the recording is
  // dropped (the solvers launch the next sweep before they wait), and neither
  // its executable graph nor the events its nodes record may be destroyed
  // before it has finished
  mutable hipStream_t launched = nullptr;
  bool valid() const { return !items.empty(); }
  void clear() {
    if (launched && (!items.empty() || !timers.empty())) (void)hipStreamSynchronize(launched);
    launched = nullptr;
    for (auto& it : items)
      if (it.exec) (void)hipGraphExecDestroy(it.exec);
    items.clear();
    if (pending)
      for (auto& t : timers) (void)hipEventSynchronize(t.b);
    pending = false;
    for (auto& t : timers) {
      (void)hipEventDestroy(t.a);
      (void)hipEventDestroy(t.b);
    }
    timers.clear();
  }
  Program() = default;
  Program(const Program&) = delete;
  Program& operator=(const Program&) = delete;
  ~Program() { clear(); }
};

class Engine {
 public:
  explicit Engine(int device);
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  hipStream_t stream = nullptr;  // the engine's own stream unless the caller sets one
  Prec prec = Prec::FP64;
  // Incremented whenever a device buffer that recorded launches may point to
  // is allocated, moved or freed (tensors, plans, workspaces, cache entries).
  uint64_t epoch = 1;
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
  // zero(t) for every tensor, plus extra[0 .. extra_n) when given, in one launch
  void zero_many(const std::vector<Tensor*>& ts, double* extra = nullptr, int64_t extra_n = 0);

  // --- terms
  void term(const std::string& spec, double scale = 1.0);
  // the packed-GEMM shape and flops the term would run with (plans it, launches nothing)
  GemmStats term_shape(const std::string& spec);
  void terms(const char* const* specs, int n, double scale = 1.0);

  // --- expansion cache
  // Operand matrices expanded from the named tensors are kept and reused by
  // later terms (directly or transposed, with the sign of the slot
  // arrangement) until the next call, which invalidates every entry.  The
  // caller guarantees that the named tensors do not change in between.
  void cache_operands(const std::vector<std::string>& names);
  size_t cache_bytes() const;

  // --- statistics (per-term algorithmic flops of the GEMMs issued)
  bool record = false;
  std::vector<GemmStats> stats;

  // Deferred GEMMs: while `sink` is set, a term issues its expansions and
  // hands its GEMM (default tile, no split-K) and the rest of the term (the
  // fold) to the sink instead of running them.  The caller runs the GEMMs
  // (for instance one grouped launch over several engines' terms) and then
  // the deferred rests in order, before this engine issues its next term.
  struct GemmSink {
    std::vector<GemmArgs> gemms;
    std::vector<std::function<void()>> after;
  };
  GemmSink* sink = nullptr;

  // --- a second lane.  fork_mark() notes the main stream's current point;
  // terms issued between begin_side() and end_side() run on a side stream
  // (with its own workspaces) that starts from that point, concurrently with
  // whatever the main stream runs after it; join_side() makes the main stream
  // wait for the side lane.  Expansion-cache entries made after the mark are
  // followed by an event, and a lane using an entry made by the other waits
  // for it.
  void fork_mark();
  void begin_side();
  void end_side();
  void join_side();

  // --- recording into a Program (stream capture into a hipGraph); nothing
  // executes while recording: replay the program to run it
  void begin_record(Program& prog);
  void end_record(Program& prog);
  void abort_record();  // after an error while recording: discard the capture
  // Launches a recorded program.  Its timers are read after the launch, or,
  // with defer, at the next replay or flush_timers (the host does not wait).
  void replay(const Program& prog, bool defer = false);
  void flush_timers(const Program& prog);
  bool recording() const { return rec_ != nullptr; }
  // Capture by another owner: the caller captures this engine's stream into
  // a graph of its own; while set, the engine refuses the work that cannot be
  // captured (allocations, new plans), as during its own recordings.
  void set_external_record(Program* p) { rec_ = p; }
  hipStream_t own_stream() const { return own_stream_; }

  // --- GEMM tile autotuner: with autotune on, the first host-launched GEMM of
  // each (precision, M, N, K, layout) times every tile configuration into a
  // scratch output and keeps the fastest for that shape (per engine).
  bool autotune = false;
  int tuned_tile(const GemmArgs& g);
  std::string tuned_report() const;  // JSON object: shape key -> tile label

  // --- per-kernel profiling with HIP events on `stream`; with a non-empty
  // filter only kernels whose label contains it are timed
  bool profile = false;
  std::string profile_filter;
  bool timed(const std::string& label) const {
    return profile && (profile_filter.empty() || label.find(profile_filter) != std::string::npos);
  }
  void prof_mark(const std::string& label, const std::string& spec, double flops, double bytes, hipEvent_t a,
                 hipEvent_t b);
  hipEvent_t event();
  std::string profile_report();  // JSON aggregate per kernel label; clears the records
  // Runs `launch` (kernels on `stream`), timed under `label` when profiling
  // selects it: HIP events around it, or event-record nodes while recording.
  void timed_launch(const std::string& label, const std::string& spec, double flops, double bytes,
                    const std::function<void()>& launch);

  // workspace sizes (bytes) currently held
  size_t workspace_bytes() const {
    size_t b = 0;
    for (size_t x : ws_bytes_) b += x;
    return b;
  }
  void* workspace(int slot, size_t bytes);

  // device buffers for tables
 private:
  struct Plan;
  std::map<std::string, std::unique_ptr<Tensor>> reg_;
  std::map<std::string, std::shared_ptr<Plan>> plans_;
  hipStream_t own_stream_ = nullptr;
  Program* rec_ = nullptr;
  struct CacheEntry {
    std::string tensor;
    void* hi = nullptr;
    void* lo = nullptr;
    size_t bytes = 0;  // per buffer
    int64_t ld = 0;    // row stride of the stored matrix (elements)
    int sign = 1;      // stored matrix = sign * canonical matrix
    bool valid = false;
    int lane = 0;                 // lane that made the current contents
    hipEvent_t ready = nullptr;   // recorded after that expansion
    bool ready_set = false;       // made after the fork mark: consumers on the other lane wait
    uint64_t fork_id = 0;         // fork cycle in which it was made
  };
  // lanes: `stream` and ws_ belong to the lane being issued to; other_* to the
  // other one (swapped by begin_side / end_side)
  hipStream_t side_stream_ = nullptr, other_stream_ = nullptr;
  hipEvent_t fork_ev_ = nullptr, join_ev_ = nullptr;
  int lane_ = 0;
  uint64_t fork_id_ = 0;  // counts fork_mark() calls
  bool side_open_ = false, fork_marked_ = false;
  void* other_ws_[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t other_ws_bytes_[7] = {0, 0, 0, 0, 0, 0, 0};
  void swap_lanes();
  std::map<std::string, CacheEntry> ecache_;
  std::vector<std::string> cacheable_;
  bool is_cacheable(const std::string& name) const {
    return std::find(cacheable_.begin(), cacheable_.end(), name) != cacheable_.end();
  }
  void* ws_[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t ws_bytes_[7] = {0, 0, 0, 0, 0, 0, 0};
  std::map<std::string, std::pair<int, std::string>> tuned_;  // shape key -> (tile, label)
  uint32_t* d_binom_ = nullptr;
  uint8_t* d_dec_[kMaxGroup + 1] = {};
  struct ProfRec {
    std::string label, spec;
    double flops, bytes;
    hipEvent_t a, b;
    float ms = -1.0f;  // already read (graph timers), else from the events
  };
  std::vector<ProfRec> prof_;
  std::vector<hipEvent_t> evpool_;
  size_t evnext_ = 0;
  std::shared_ptr<Plan> plan(const std::string& spec);
  void execute(const Plan& p, double scale);
};

// Expansion cache enabled for the named tensors for the lifetime of the scope.
struct CacheScope {
  Engine& e;
  CacheScope(Engine& en, const std::vector<std::string>& names) : e(en) { e.cache_operands(names); }
  ~CacheScope() { e.cache_operands({}); }
  CacheScope(const CacheScope&) = delete;
  CacheScope& operator=(const CacheScope&) = delete;
};

}  // namespace fno

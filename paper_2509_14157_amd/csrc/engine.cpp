// Contraction planner and executor (host side).
#include "engine.hpp"

#include <array>
#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <cctype>
#include <cstring>
#include <functional>
#include <sstream>

namespace fno {

// ------------------------------------------------------------------ tables
static void colex_tuples(int n, int g, std::vector<uint8_t>& out) {
  // colex order: by largest element, then recursively
  std::vector<int> cur(g);
  std::function<void(int, int)> rec = [&](int pos, int limit) {
    // choose cur[pos] < limit, cur[pos] is the largest among positions <= pos
    for (int x = pos; x < limit; ++x) {
      cur[pos] = x;
      if (pos == 0) {
        for (int t = 0; t < g; ++t) out.push_back((uint8_t)cur[t]);
      } else {
        rec(pos - 1, x);
      }
    }
  };
  rec(g - 1, n);
}

Engine::Engine(int dev) : device(dev) {
  FNO_HIP(hipSetDevice(device));
  FNO_HIP(hipStreamCreate(&own_stream_));
  stream = own_stream_;
  std::vector<uint32_t> b(kBinomN * (kMaxGroup + 1));
  for (int n = 0; n < kBinomN; ++n)
    for (int k = 0; k <= kMaxGroup; ++k) b[n * (kMaxGroup + 1) + k] = (uint32_t)binom_host(n, k);
  FNO_HIP(hipMalloc(&d_binom_, b.size() * sizeof(uint32_t)));
  FNO_HIP(hipMemcpy(d_binom_, b.data(), b.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  tables.binom = d_binom_;
  const int maxn[kMaxGroup + 1] = {0, 0, 256, 128, 64};
  for (int g = 2; g <= kMaxGroup; ++g) {
    std::vector<uint8_t> t;
    colex_tuples(maxn[g], g, t);
    // self-check of the colex rank formula
    for (size_t i = 0; i < t.size() / g; i += 997) {
      uint64_t r = 0;
      for (int s = 0; s < g; ++s) r += binom_host(t[i * g + s], s + 1);
      FNO_REQUIRE(r == i, kEDEVICE, "colex table self-check failed");
    }
    FNO_HIP(hipMalloc(&d_dec_[g], t.size()));
    FNO_HIP(hipMemcpy(d_dec_[g], t.data(), t.size(), hipMemcpyHostToDevice));
    tables.dec[g] = d_dec_[g];
    tables.dec_max_n[g] = maxn[g];
  }
  tables.dec_max_n[1] = 1 << 30;
}

Engine::~Engine() {
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (auto& kv : reg_)
    if (kv.second->owner && kv.second->d) (void)hipFree(kv.second->d);
  for (int i = 0; i < 7; ++i) {
    if (ws_[i]) (void)hipFree(ws_[i]);
    if (other_ws_[i]) (void)hipFree(other_ws_[i]);
  }
  for (auto ev : evpool_) (void)hipEventDestroy(ev);
  for (auto& kv : ecache_) {
    if (kv.second.hi) (void)hipFree(kv.second.hi);
    if (kv.second.lo) (void)hipFree(kv.second.lo);
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  }
  if (fork_ev_) (void)hipEventDestroy(fork_ev_);
  if (join_ev_) (void)hipEventDestroy(join_ev_);
  if (side_stream_) (void)hipStreamDestroy(side_stream_);
  if (d_binom_) (void)hipFree(d_binom_);
  for (int g = 0; g <= kMaxGroup; ++g)
    if (d_dec_[g]) (void)hipFree(d_dec_[g]);
  if (own_stream_) (void)hipStreamDestroy(own_stream_);
}

// ------------------------------------------------------------------ lanes
void Engine::swap_lanes() {
  std::swap(stream, other_stream_);
  for (int i = 0; i < 7; ++i) {
    std::swap(ws_[i], other_ws_[i]);
    std::swap(ws_bytes_[i], other_ws_bytes_[i]);
  }
  lane_ = 1 - lane_;
}

void Engine::fork_mark() {
  FNO_REQUIRE(lane_ == 0 && !side_open_ && !fork_marked_, kEINVAL, "side lane already forked");
  if (!side_stream_) {
    FNO_REQUIRE(!rec_, kEINVAL, "side lane created while recording");
    FNO_HIP(hipStreamCreate(&side_stream_));
    FNO_HIP(hipEventCreateWithFlags(&fork_ev_, hipEventDisableTiming));
    FNO_HIP(hipEventCreateWithFlags(&join_ev_, hipEventDisableTiming));
  }
  FNO_HIP(hipEventRecord(fork_ev_, stream));
  fork_marked_ = true;
  ++fork_id_;
}

void Engine::begin_side() {
  FNO_REQUIRE(lane_ == 0 && !side_open_, kEINVAL, "side lane already open");
  if (!fork_marked_) fork_mark();
  FNO_HIP(hipStreamWaitEvent(side_stream_, fork_ev_, 0));
  other_stream_ = side_stream_;
  swap_lanes();
  side_open_ = true;
}

void Engine::end_side() {
  FNO_REQUIRE(lane_ == 1, kEINVAL, "not issuing to the side lane");
  FNO_HIP(hipEventRecord(join_ev_, stream));
  swap_lanes();
}

void Engine::join_side() {
  if (lane_ == 1) end_side();
  fork_marked_ = false;
  if (!side_open_) return;
  side_open_ = false;
  FNO_HIP(hipStreamWaitEvent(stream, join_ev_, 0));
}

// ------------------------------------------------------------------ recording
void Engine::begin_record(Program& prog) {
  FNO_REQUIRE(rec_ == nullptr, kEINVAL, "nested recording");
  FNO_REQUIRE(stream != nullptr, kEINVAL, "recording needs a non-null stream");
  prog.clear();
  prog.epoch = epoch;
  prog.prec = (int)prec;
  prog.profiled = profile;
  prog.filter = profile_filter;
  rec_ = &prog;
  FNO_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
}

void Engine::end_record(Program& prog) {
  FNO_REQUIRE(rec_ == &prog, kEINVAL, "not recording this program");
  hipGraph_t g = nullptr;
  hipError_t err = hipStreamEndCapture(stream, &g);
  rec_ = nullptr;
  FNO_HIP(err);
  size_t nodes = 0;
  FNO_HIP(hipGraphGetNodes(g, nullptr, &nodes));
  if (nodes > 0) {
    Program::Item it;
    FNO_HIP(hipGraphInstantiate(&it.exec, g, nullptr, nullptr, 0));
    prog.items.push_back(std::move(it));
  }
  FNO_HIP(hipGraphDestroy(g));
  // a recording is only valid if nothing was (re)allocated while it ran
  if (prog.epoch != epoch) prog.clear();
}

void Engine::abort_record() {
  if (!rec_) return;
  Program* prog = rec_;
  rec_ = nullptr;
  hipGraph_t g = nullptr;
  (void)hipStreamEndCapture(stream, &g);
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  prog->clear();
}

void Engine::flush_timers(const Program& prog) {
  if (!prog.pending) return;
  for (const auto& t : prog.timers) FNO_HIP(hipEventSynchronize(t.b));
  for (const auto& t : prog.timers) {
    float ms = 0;
    FNO_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    prof_.push_back({t.label, t.spec, t.flops, t.bytes, nullptr, nullptr, ms});
  }
  prog.pending = false;
}

void Engine::replay(const Program& prog, bool defer) {
  // the event nodes are re-recorded by this replay: read the last one's first
  flush_timers(prog);
  prog.launched = stream;
  for (auto& it : prog.items) FNO_HIP(hipGraphLaunch(it.exec, stream));
  if (!prog.timers.empty()) {
    prog.pending = true;
    if (!defer) flush_timers(prog);
  }
}

void* Engine::workspace(int slot, size_t bytes) {
  if (bytes > ws_bytes_[slot]) {
    FNO_REQUIRE(!rec_, kEINVAL, "workspace growth while recording");
    ++epoch;
    if (ws_[slot]) {
      FNO_HIP(hipStreamSynchronize(stream));
      FNO_HIP(hipFree(ws_[slot]));
      ws_[slot] = nullptr;
      ws_bytes_[slot] = 0;
    }
    size_t b = std::max(bytes, (size_t)(1 << 20));
    FNO_HIP(hipMalloc(&ws_[slot], b));
    ws_bytes_[slot] = b;
  }
  return ws_[slot];
}

// ------------------------------------------------------------------ profiling
hipEvent_t Engine::event() {
  if (evnext_ == evpool_.size()) {
    hipEvent_t ev;
    FNO_HIP(hipEventCreate(&ev));
    evpool_.push_back(ev);
  }
  return evpool_[evnext_++];
}

void Engine::prof_mark(const std::string& label, const std::string& spec, double flops, double bytes, hipEvent_t a,
                       hipEvent_t b) {
  prof_.push_back({label, spec, flops, bytes, a, b});
}

void Engine::timed_launch(const std::string& label, const std::string& spec, double flops, double bytes,
                          const std::function<void()>& launch) {
  if (!timed(label)) {
    launch();
    return;
  }
  if (rec_) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FNO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      throw Error(kEDEVICE, "hipEventCreate failed");
    }
    rec_->timers.push_back({label, spec, flops, bytes, e0, e1});
    FNO_HIP(hipEventRecordWithFlags(e0, stream, hipEventRecordExternal));
    launch();
    FNO_HIP(hipEventRecordWithFlags(e1, stream, hipEventRecordExternal));
    return;
  }
  hipEvent_t e0 = event();
  FNO_HIP(hipEventRecord(e0, stream));
  launch();
  hipEvent_t e1 = event();
  FNO_HIP(hipEventRecord(e1, stream));
  prof_mark(label, spec, flops, bytes, e0, e1);
}

std::string Engine::profile_report() {
  FNO_HIP(hipStreamSynchronize(stream));
  if (side_stream_) FNO_HIP(hipStreamSynchronize(side_stream_));
  struct Agg {
    int64_t n = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::map<std::string, Agg> agg;
  std::map<std::string, Agg> per_term;
  for (auto& r : prof_) {
    float ms = r.ms;
    if (ms < 0) FNO_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    Agg& a = agg[r.label];
    a.n++;
    a.ms += ms;
    a.flops += r.flops;
    a.bytes += r.bytes;
    Agg& t = per_term[r.spec + " @ " + r.label];
    t.n++;
    t.ms += ms;
    t.flops += r.flops;
    t.bytes += r.bytes;
  }
  auto esc = [](const std::string& s) {
    std::string o;
    for (char c : s) {
      if (c == '"' || c == '\\') o += '\\';
      o += c;
    }
    return o;
  };
  std::string js = "{\"kernels\": [";
  bool first = true;
  for (auto& kv : agg) {
    char buf[256];
    snprintf(buf, sizeof(buf), "\"launches\": %lld, \"total_ms\": %.6f, \"flops\": %.6e, \"bytes\": %.6e}",
             (long long)kv.second.n, kv.second.ms, kv.second.flops, kv.second.bytes);
    js += std::string(first ? "" : ", ") + "{\"name\": \"" + esc(kv.first) + "\", " + buf;
    first = false;
  }
  js += "], \"terms\": [";
  first = true;
  for (auto& kv : per_term) {
    char buf[256];
    snprintf(buf, sizeof(buf), "\"launches\": %lld, \"total_ms\": %.6f, \"flops\": %.6e, \"bytes\": %.6e}",
             (long long)kv.second.n, kv.second.ms, kv.second.flops, kv.second.bytes);
    js += std::string(first ? "" : ", ") + "{\"term\": \"" + esc(kv.first) + "\", " + buf;
    first = false;
  }
  js += "], \"tuned\": " + tuned_report() + "}";
  prof_.clear();
  evnext_ = 0;
  return js;
}

// ------------------------------------------------------------------ tensors
int64_t Engine::spec_size(const std::string& spec, const SpaceSizes& sz) {
  std::stringstream ss(spec);
  std::string tok;
  int64_t e = 1;
  while (std::getline(ss, tok, ',')) {
    if (tok.empty()) continue;
    auto it = sz.n.find(tok[0]);
    FNO_REQUIRE(it != sz.n.end(), kEINVAL, std::string("unknown space ") + tok[0]);
    e *= (int64_t)binom_host(it->second, (int)tok.size());
  }
  return e;
}

Tensor* Engine::create(const std::string& name, const std::string& spec, const SpaceSizes& sz, double* external) {
  FNO_REQUIRE(!rec_, kEINVAL, "tensor creation while recording");
  ++epoch;
  FNO_REQUIRE(!reg_.count(name), kEINVAL, "tensor exists: " + name);
  auto t = std::make_unique<Tensor>();
  t->name = name;
  std::stringstream ss(spec);
  std::string tok;
  while (std::getline(ss, tok, ',')) {
    if (tok.empty()) continue;
    Group g;
    g.g = (int)tok.size();
    for (char c : tok) FNO_REQUIRE(c == tok[0], kEINVAL, "mixed spaces in group " + tok);
    auto it = sz.n.find(tok[0]);
    FNO_REQUIRE(it != sz.n.end(), kEINVAL, std::string("unknown space ") + tok[0]);
    g.n = g.ext = it->second;
    FNO_REQUIRE(g.g <= kMaxGroup, kEINVAL, "group too large");
    if (g.g > 1) FNO_REQUIRE(g.n <= tables.dec_max_n[g.g], kEINVAL, "index range too large for packed group");
    t->groups.push_back(g);
  }
  FNO_REQUIRE(t->nslots() <= kMaxSlots && (int)t->groups.size() <= kMaxGroups, kEINVAL, "tensor rank too large");
  int64_t e = 1;
  int slot = 0;
  for (auto& g : t->groups) {
    e *= g.storage();
    std::vector<int> sl;
    for (int k = 0; k < g.g; ++k) sl.push_back(slot++);
    t->sym.push_back(sl);
  }
  t->elems = e;
  if (external) {
    t->d = external;
    t->owner = false;
  } else {
    if (e > 0) {
      FNO_HIP(hipMalloc(&t->d, (size_t)e * sizeof(double)));
      launch_fill(t->d, 0.0, e, stream);
    }
    t->owner = true;
  }
  Tensor* p = t.get();
  reg_[name] = std::move(t);
  return p;
}

Tensor* Engine::view(const std::string& name, Tensor* parent, const std::vector<std::pair<int, int>>& ranges) {
  FNO_REQUIRE(parent != nullptr, kEINVAL, "view of null tensor");
  FNO_REQUIRE(ranges.size() == parent->groups.size(), kEINVAL, "view rank mismatch");
  auto t = std::make_unique<Tensor>(*parent);
  t->name = name;
  t->owner = false;
  for (size_t q = 0; q < ranges.size(); ++q) {
    Group& g = t->groups[q];
    int off = ranges[q].first, n = ranges[q].second;
    if (g.g > 1) {
      FNO_REQUIRE(off == 0 && n == g.ext, kEINVAL, "packed groups cannot be sliced");
      continue;
    }
    FNO_REQUIRE(off >= 0 && off + n <= g.ext, kEINVAL, "view out of range");
    g.off = parent->groups[q].off + off;
    g.n = n;
  }
  // a declared antisymmetric slot set survives the view only if all its
  // slots see the same index range
  {
    std::vector<int> slot_grp, slot_first(t->nslots());
    std::vector<std::pair<int, int>> rng;
    int s = 0;
    for (size_t q = 0; q < t->groups.size(); ++q)
      for (int k = 0; k < t->groups[q].g; ++k, ++s) rng.push_back({t->groups[q].off, t->groups[q].n});
    std::vector<std::vector<int>> sym;
    for (auto& set : t->sym) {
      bool same = true;
      for (int sl : set) same = same && rng[sl] == rng[set[0]];
      if (same) {
        sym.push_back(set);
      } else {
        for (int sl : set) sym.push_back({sl});
      }
    }
    t->sym = sym;
  }
  Tensor* p = t.get();
  auto it = reg_.find(name);
  if (it != reg_.end()) {
    FNO_REQUIRE(!it->second->owner, kEINVAL, "cannot replace an owning tensor by a view: " + name);
    // invalidate plans that captured the old view
    for (auto pit = plans_.begin(); pit != plans_.end();)
      if (pit->first.find(name) != std::string::npos)
        pit = plans_.erase(pit);
      else
        ++pit;
  }
  reg_[name] = std::move(t);
  return p;
}

Tensor* Engine::get(const std::string& name) const {
  auto it = reg_.find(name);
  FNO_REQUIRE(it != reg_.end(), kEINVAL, "unknown tensor " + name);
  return it->second.get();
}

void Engine::set_sym(Tensor* t, const std::vector<std::vector<int>>& sym) {
  std::vector<int> seen(t->nslots(), 0);
  for (auto& set : sym)
    for (int sl : set) {
      FNO_REQUIRE(sl >= 0 && sl < t->nslots() && !seen[sl], kEINVAL, "bad symmetry partition");
      seen[sl] = 1;
    }
  for (int x : seen) FNO_REQUIRE(x, kEINVAL, "symmetry partition must cover every slot");
  t->sym = sym;
}

void Engine::drop(const std::string& name) {
  FNO_REQUIRE(!rec_, kEINVAL, "tensor release while recording");
  ++epoch;
  auto it = reg_.find(name);
  if (it == reg_.end()) return;
  if (it->second->owner && it->second->d) {
    FNO_HIP(hipStreamSynchronize(stream));
    FNO_HIP(hipFree(it->second->d));
  }
  reg_.erase(it);
  for (auto cit = ecache_.begin(); cit != ecache_.end();)
    if (cit->second.tensor == name) {
      FNO_HIP(hipStreamSynchronize(stream));
      if (cit->second.hi) FNO_HIP(hipFree(cit->second.hi));
      if (cit->second.lo) FNO_HIP(hipFree(cit->second.lo));
      cit = ecache_.erase(cit);
    } else {
      ++cit;
    }
  for (auto pit = plans_.begin(); pit != plans_.end();)
    if (pit->first.find(name) != std::string::npos)
      pit = plans_.erase(pit);
    else
      ++pit;
}

void Engine::zero(Tensor* t) {
  FNO_REQUIRE(t->full_view(), kEINVAL, "zero() needs a whole tensor");
  launch_fill(t->d, 0.0, t->elems, stream);
}

void Engine::zero_many(const std::vector<Tensor*>& ts, double* extra, int64_t extra_n) {
  std::vector<double*> p;
  std::vector<int64_t> n;
  if (extra) {
    p.push_back(extra);
    n.push_back(extra_n);
  }
  for (Tensor* t : ts) {
    FNO_REQUIRE(t->full_view(), kEINVAL, "zero() needs a whole tensor");
    p.push_back(t->d);
    n.push_back(t->elems);
  }
  launch_zero_many(p.data(), n.data(), (int)p.size(), stream);
}

// ------------------------------------------------------------------ planning
struct Engine::Plan {
  std::string spec;
  Tensor *out = nullptr, *A = nullptr, *B = nullptr;
  double alpha = 1;
  MatDim M{}, N{}, K{};
  bool a_direct = false, a_kfast = true;
  int64_t lda = 0;
  OperandDesc ad{};
  bool b_direct = false, b_nfast = true;
  int64_t ldb = 0;
  OperandDesc bd{};
  bool x_direct = false;
  bool copy_direct = false;  // single operand expanded straight into the output
  OperandDesc od{};
  MatDim odims{};
  FoldCombos fc{};
  double flops = 0;
  Prec prec = Prec::FP64;
  // expansion-cache keys of A (M x K) and B (K x N), and the parity of this
  // term's slot arrangement relative to the key's canonical one (direct and
  // transposed use)
  bool a_cache = false, b_cache = false;
  std::string a_key, a_keyT, b_key, b_keyT;
  int a_sign = 1, a_signT = 1, b_sign = 1, b_signT = 1;
  // table-driven expansion / fold (device tables owned by the plan)
  bool a_tab_ok = false, b_tab_ok = false, f_tab_ok = false;
  ExpandTab a_tab{}, b_tab{};
  FoldTab f_tab{};
  std::vector<void*> bufs;
  ~Plan() {
    for (void* p : bufs) (void)hipFree(p);
  }
};

namespace {
// Expansion tables of operand `od` (storage letter groups `st`) into a
// rows x cols matrix; false when the operand has more straddling groups than
// the kernel supports.
bool build_expand_tab(const IndexTables& tb, const OperandDesc& od, const std::vector<std::vector<int>>& st,
                      const MatDim& rows, const MatDim& cols, ExpandTab& t, std::vector<void*>& bufs,
                      hipStream_t s) {
  auto in_dim = [](const MatDim& d, int l) {
    for (int q = 0; q < d.ngroups; ++q)
      for (int k = 0; k < d.grp[q].g; ++k)
        if (d.grp[q].letter[k] == l) return q;
    return -1;
  };
  unsigned row_mask = 0, col_mask = 0;
  std::vector<int> mixed;
  for (size_t q = 0; q < st.size(); ++q) {
    bool r = false, c = false;
    for (int l : st[q]) {
      if (in_dim(rows, l) >= 0) r = true;
      else if (in_dim(cols, l) >= 0) c = true;
      else return false;
    }
    if (r && c)
      mixed.push_back((int)q);
    else if (r)
      row_mask |= 1u << q;
    else
      col_mask |= 1u << q;
  }
  if ((int)mixed.size() > kMaxMixed) return false;
  auto dalloc = [&](size_t bytes) {
    void* p = nullptr;
    FNO_HIP(hipMalloc(&p, std::max<size_t>(bytes, 8)));
    bufs.push_back(p);
    return p;
  };
  t = ExpandTab{};
  t.rows = rows.size;
  t.cols = cols.size;
  t.ld = cols.size;
  int64_t* ro = (int64_t*)dalloc(rows.size * 8);
  int8_t* rs = (int8_t*)dalloc(rows.size);
  int64_t* co = (int64_t*)dalloc(cols.size * 8);
  int8_t* cs = (int8_t*)dalloc(cols.size);
  OperandDesc rod = od, cod = od;
  rod.base = od.base;  // the view origin is carried by the row table
  cod.base = 0;
  launch_dim_table(tb, rod, rows, row_mask, ro, rs, s);
  launch_dim_table(tb, cod, cols, col_mask, co, cs, s);
  t.row_off = ro;
  t.row_sign = rs;
  t.col_off = co;
  t.col_sign = cs;
  t.nmixed = (int)mixed.size();
  for (int m = 0; m < t.nmixed; ++m) {
    const int q = mixed[m];
    unsigned rdm = 0, cdm = 0;
    MatDim pr{}, pc{};
    pr.size = pc.size = 1;
    for (int g = 0; g < rows.ngroups; ++g) {
      bool inq = false;
      for (int l : st[q]) inq |= in_dim(rows, l) == g;
      if (inq) {
        rdm |= 1u << g;
        pr.grp[pr.ngroups++] = rows.grp[g];
        pr.size *= rows.grp[g].count;
      }
    }
    for (int g = 0; g < cols.ngroups; ++g) {
      bool inq = false;
      for (int l : st[q]) inq |= in_dim(cols, l) == g;
      if (inq) {
        cdm |= 1u << g;
        pc.grp[pc.ngroups++] = cols.grp[g];
        pc.size *= cols.grp[g].count;
      }
    }
    int32_t* rsub = (int32_t*)dalloc(rows.size * 4);
    int32_t* csub = (int32_t*)dalloc(cols.size * 4);
    int64_t* to = (int64_t*)dalloc(pr.size * pc.size * 8);
    int8_t* ts = (int8_t*)dalloc(pr.size * pc.size);
    launch_sub_index(tb, rows, rdm, rsub, s);
    launch_sub_index(tb, cols, cdm, csub, s);
    launch_mixed_table(tb, od, q, pr, pc, to, ts, s);
    t.ncsub[m] = pc.size;
    t.row_sub[m] = rsub;
    t.col_sub[m] = csub;
    t.tab_off[m] = to;
    t.tab_sign[m] = ts;
  }
  return true;
}
}  // namespace

namespace {

struct Parsed {
  std::string out, A, B;
  std::string lo, la, lb;
  double coef = 1;
};

void skip_ws(const std::string& s, size_t& i) {
  while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
}

std::string ident(const std::string& s, size_t& i) {
  skip_ws(s, i);
  size_t j = i;
  while (j < s.size() && (std::isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
  FNO_REQUIRE(j > i, kEINVAL, "expected a name in term: " + s);
  std::string r = s.substr(i, j - i);
  i = j;
  return r;
}

std::string bracket(const std::string& s, size_t& i) {
  skip_ws(s, i);
  FNO_REQUIRE(i < s.size() && s[i] == '[', kEINVAL, "expected [ in term: " + s);
  size_t j = s.find(']', i);
  FNO_REQUIRE(j != std::string::npos, kEINVAL, "expected ] in term: " + s);
  std::string r = s.substr(i + 1, j - i - 1);
  i = j + 1;
  return r;
}

Parsed parse(const std::string& s) {
  Parsed p;
  size_t i = 0;
  p.out = ident(s, i);
  p.lo = bracket(s, i);
  skip_ws(s, i);
  double sign = 1;
  if (s.compare(i, 2, "+=") == 0)
    sign = 1;
  else if (s.compare(i, 2, "-=") == 0)
    sign = -1;
  else
    FNO_REQUIRE(false, kEINVAL, "expected += or -= in term: " + s);
  i += 2;
  skip_ws(s, i);
  // optional coefficient
  size_t j = i;
  while (j < s.size() && (std::isdigit((unsigned char)s[j]) || s[j] == '.' || s[j] == '-' || s[j] == '/'))
    ++j;
  if (j > i) {
    std::string c = s.substr(i, j - i);
    size_t sl = c.find('/');
    if (sl != std::string::npos)
      p.coef = std::stod(c.substr(0, sl)) / std::stod(c.substr(sl + 1));
    else
      p.coef = std::stod(c);
    i = j;
    skip_ws(s, i);
    FNO_REQUIRE(i < s.size() && s[i] == '*', kEINVAL, "expected * after coefficient: " + s);
    ++i;
  }
  p.coef *= sign;
  p.A = ident(s, i);
  p.la = bracket(s, i);
  skip_ws(s, i);
  if (i < s.size() && s[i] == '*') {
    ++i;
    p.B = ident(s, i);
    p.lb = bracket(s, i);
  }
  skip_ws(s, i);
  FNO_REQUIRE(i == s.size(), kEINVAL, "trailing text in term: " + s);
  return p;
}

// letters of a tensor grouped by its storage groups
std::vector<std::vector<int>> letter_groups(const Tensor* t, const std::vector<int>& ids) {
  std::vector<std::vector<int>> out;
  size_t s = 0;
  for (auto& g : t->groups) {
    std::vector<int> v;
    for (int k = 0; k < g.g; ++k) v.push_back(ids[s++]);
    out.push_back(v);
  }
  return out;
}

// letters of a tensor grouped by its antisymmetry partition
std::vector<std::vector<int>> letter_syms(const Tensor* t, const std::vector<int>& ids) {
  std::vector<std::vector<int>> out;
  for (auto& set : t->sym) {
    std::vector<int> v;
    for (int sl : set) v.push_back(ids[sl]);
    out.push_back(v);
  }
  return out;
}

int64_t factorial(int n) {
  int64_t r = 1;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

int perm_sign(const std::vector<int>& p) {
  std::vector<int> q = p;
  int s = 1;
  for (size_t i = 0; i < q.size(); ++i)
    while (q[i] != (int)i) {
      std::swap(q[i], q[q[i]]);
      s = -s;
    }
  return s;
}

// Canonical description of the matrix a packed operand expands into: for each
// row group and each column group, the storage group it is cut from and its
// size.  Two expansions with the same description hold the same values up to
// the parity of where their letters sit inside the antisymmetric storage
// groups; `sign` is that parity relative to the order (rows first, then
// columns, each by group and position), `signT` relative to (columns first).
struct CanonKey {
  bool ok = false;
  std::string key, keyT;
  int sign = 1, signT = 1;
};

CanonKey canon_key(const Tensor* t, const std::vector<int>& ids, const MatDim& rows, const MatDim& cols, Prec prec) {
  CanonKey ck;
  std::vector<std::vector<int>> st;
  int s = 0;
  for (auto& g : t->groups) {
    std::vector<int> v;
    for (int k = 0; k < g.g; ++k) v.push_back(s++);
    st.push_back(v);
  }
  if (t->sym != st) return ck;  // only packed antisymmetric tensors
  const int ns = s;
  std::vector<int> grp_of(ns);
  for (size_t q = 0; q < st.size(); ++q)
    for (int x : st[q]) grp_of[x] = (int)q;
  std::vector<std::array<int, 3>> where(ns, {-1, -1, -1});
  const MatDim* side[2] = {&rows, &cols};
  std::string desc[2];
  for (int sd = 0; sd < 2; ++sd)
    for (int q = 0; q < side[sd]->ngroups; ++q) {
      const DimGroup& G = side[sd]->grp[q];
      int src = -1;
      for (int k = 0; k < G.g; ++k) {
        int slot = -1;
        for (int x = 0; x < ns; ++x)
          if (ids[x] == G.letter[k]) slot = x;
        if (slot < 0) return ck;
        if (src < 0) src = grp_of[slot];
        if (grp_of[slot] != src) return ck;
        where[slot] = {sd, q, k};
      }
      desc[sd] += "(" + std::to_string(src) + "," + std::to_string(G.g) + ")";
    }
  for (auto& w : where)
    if (w[0] < 0) return ck;
  auto parity = [&](bool trans) {
    int sg = 1;
    for (auto& gslots : st) {
      std::vector<int> ord = gslots;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        std::array<int, 3> wa = where[a], wb = where[b];
        if (trans) {
          wa[0] = 1 - wa[0];
          wb[0] = 1 - wb[0];
        }
        return wa < wb;
      });
      std::vector<int> pos(ord.size());
      for (size_t i = 0; i < ord.size(); ++i) pos[i] = ord[i] - gslots[0];
      sg *= perm_sign(pos);
    }
    return sg;
  };
  char ptr[32];
  std::snprintf(ptr, sizeof(ptr), "%p", (const void*)t->d);
  const std::string head = t->name + "@" + ptr + "#" + std::to_string((int)prec) + "|";
  ck.key = head + desc[0] + "|" + desc[1];
  ck.keyT = head + desc[1] + "|" + desc[0];
  ck.sign = parity(false);
  ck.signT = parity(true);
  ck.ok = true;
  return ck;
}

}  // namespace

GemmStats Engine::term_shape(const std::string& spec) {
  auto p = plan(spec);
  return {spec, p->M.size, p->N.size, p->K.size, p->flops};
}

std::shared_ptr<Engine::Plan> Engine::plan(const std::string& spec) {
  // zero-copy decisions depend on the precision: plans are cached per precision
  const std::string key = spec + "#" + std::to_string((int)prec);
  auto it = plans_.find(key);
  if (it != plans_.end()) return it->second;
  Parsed ps = parse(spec);
  FNO_REQUIRE(!rec_, kEINVAL, "new contraction plan while recording");
  ++epoch;
  auto P = std::make_shared<Plan>();
  P->spec = spec;
  P->out = get(ps.out);
  P->A = get(ps.A);
  P->B = ps.B.empty() ? nullptr : get(ps.B);
  FNO_REQUIRE((int)ps.lo.size() == P->out->nslots(), kEINVAL, "letter count mismatch (out): " + spec);
  FNO_REQUIRE((int)ps.la.size() == P->A->nslots(), kEINVAL, "letter count mismatch (A): " + spec);
  if (P->B) FNO_REQUIRE((int)ps.lb.size() == P->B->nslots(), kEINVAL, "letter count mismatch (B): " + spec);

  // letter ids and extents
  std::vector<char> letters;
  auto id_of = [&](char c) {
    auto f = std::find(letters.begin(), letters.end(), c);
    if (f != letters.end()) return (int)(f - letters.begin());
    letters.push_back(c);
    return (int)letters.size() - 1;
  };
  std::vector<int> io, ia, ib;
  for (char c : ps.lo) io.push_back(id_of(c));
  for (char c : ps.la) ia.push_back(id_of(c));
  for (char c : ps.lb) ib.push_back(id_of(c));
  const int L = (int)letters.size();
  FNO_REQUIRE(L <= kMaxLetters, kEINVAL, "too many letters: " + spec);
  std::vector<int> ext(L, -1);
  auto note_ext = [&](const Tensor* t, const std::vector<int>& ids) {
    size_t s = 0;
    for (auto& g : t->groups)
      for (int k = 0; k < g.g; ++k, ++s) {
        int l = ids[s];
        if (ext[l] < 0) ext[l] = g.n;
        FNO_REQUIRE(ext[l] == g.n, kEINVAL, "extent mismatch of letter " + std::string(1, letters[l]) + ": " + spec);
      }
  };
  note_ext(P->out, io);
  note_ext(P->A, ia);
  if (P->B) note_ext(P->B, ib);
  auto in = [](const std::vector<int>& v, int l) { return std::find(v.begin(), v.end(), l) != v.end(); };
  for (int l = 0; l < L; ++l) {
    int c = in(io, l) + in(ia, l) + in(ib, l);
    FNO_REQUIRE(c == 2 || (c == 1 && in(io, l) && !P->B), kEINVAL,
                "each letter must appear in exactly two tensors: " + spec);
    FNO_REQUIRE(!(in(io, l) && !in(ia, l) && !in(ib, l)), kEINVAL, "free output letter: " + spec);
  }
  for (int l = 0; l < L; ++l) FNO_REQUIRE(std::count(io.begin(), io.end(), l) <= 1, kEINVAL, "repeated letter");

  // output symmetry is always its storage packing; operands may carry more
  auto go = letter_groups(P->out, io);
  auto ga = letter_syms(P->A, ia);
  auto ga_st = letter_groups(P->A, ia);
  std::vector<std::vector<int>> gb, gb_st;
  if (P->B) {
    gb = letter_syms(P->B, ib);
    gb_st = letter_groups(P->B, ib);
  }

  // X row groups (from A), column groups (from B), K groups (A x B)
  std::vector<std::vector<int>> mg, ngp, kg;
  for (auto& a : ga)
    for (auto& o : go) {
      std::vector<int> v;
      for (int l : a)
        if (in(o, l)) v.push_back(l);
      if (!v.empty()) mg.push_back(v);
    }
  for (auto& b : gb)
    for (auto& o : go) {
      std::vector<int> v;
      for (int l : b)
        if (in(o, l)) v.push_back(l);
      if (!v.empty()) ngp.push_back(v);
    }
  int64_t kfac = 1;
  for (auto& a : ga)
    for (auto& b : gb) {
      std::vector<int> v;
      for (int l : a)
        if (in(b, l)) v.push_back(l);
      if (!v.empty()) {
        kg.push_back(v);
        kfac *= factorial((int)v.size());
      }
    }
  auto mkdim = [&](const std::vector<std::vector<int>>& gs) {
    MatDim d{};
    FNO_REQUIRE((int)gs.size() <= kMaxGroups, kEINVAL, "too many groups: " + spec);
    d.ngroups = (int)gs.size();
    d.size = 1;
    for (size_t q = 0; q < gs.size(); ++q) {
      DimGroup& G = d.grp[q];
      G.g = (int)gs[q].size();
      FNO_REQUIRE(G.g <= kMaxGroup, kEINVAL, "group too large: " + spec);
      G.n = ext[gs[q][0]];
      if (G.g > 1) FNO_REQUIRE(G.n <= tables.dec_max_n[G.g], kEINVAL, "range too large for packed group: " + spec);
      G.count = G.g == 1 ? G.n : (int64_t)binom_host(G.n, G.g);
      for (int s = 0; s < G.g; ++s) G.letter[s] = (int8_t)gs[q][s];
      d.size *= G.count;
    }
    return d;
  };
  P->M = mkdim(mg);
  P->N = mkdim(ngp);
  P->K = mkdim(kg);
  P->odims = mkdim(go);
  P->alpha = ps.coef * (double)kfac;
  P->flops = 2.0 * (double)P->M.size * (double)P->N.size * (double)P->K.size;

  auto opdesc = [&](const Tensor* t, const std::vector<int>& ids) {
    OperandDesc d{};
    d.ngroups = (int)t->groups.size();
    d.base = t->base;
    auto st = t->strides();
    size_t s = 0;
    for (size_t q = 0; q < t->groups.size(); ++q) {
      GroupDesc& G = d.grp[q];
      G.g = t->groups[q].g;
      G.off = t->groups[q].off;
      G.stride = st[q];
      for (int k = 0; k < G.g; ++k) G.letter[k] = (int8_t)ids[s++];
    }
    return d;
  };
  P->ad = opdesc(P->A, ia);
  if (P->B) P->bd = opdesc(P->B, ib);
  P->od = opdesc(P->out, io);

  // fold combos: shuffles of every output group over its X sub-blocks
  std::vector<std::vector<std::pair<std::vector<int>, int>>> per_group;  // (src letters per slot of the group, sign)
  bool trivial = true;
  for (auto& o : go) {
    // sub-blocks: X groups inside this output group, in X-group letter order
    std::vector<std::vector<int>> subs;
    for (auto* gl : {&mg, &ngp})
      for (auto& x : *gl)
        if (in(o, x[0])) subs.push_back(x);
    const int m = (int)o.size();
    std::vector<std::pair<std::vector<int>, int>> list;
    // recursive assignment of value positions to sub-blocks
    std::vector<int> valpos(L, -1);  // letter -> value position within the group
    std::vector<bool> used(m, false);
    std::function<void(size_t)> rec = [&](size_t sb) {
      if (sb == subs.size()) {
        // permutation pi: slot position q (letter o[q]) -> value position
        std::vector<int> pi(m);
        for (int q = 0; q < m; ++q) pi[q] = valpos[o[q]];
        std::vector<int> src(m);
        for (int q = 0; q < m; ++q) src[q] = o[pi[q]];
        list.push_back({src, perm_sign(pi)});
        return;
      }
      const auto& sub = subs[sb];
      const int k = (int)sub.size();
      // choose k unused positions in increasing order
      std::vector<int> pick;
      std::function<void(int)> choose = [&](int start) {
        if ((int)pick.size() == k) {
          for (int t = 0; t < k; ++t) {
            valpos[sub[t]] = pick[t];
            used[pick[t]] = true;
          }
          rec(sb + 1);
          for (int t = 0; t < k; ++t) used[pick[t]] = false;
          return;
        }
        for (int p = start; p < m; ++p)
          if (!used[p]) {
            pick.push_back(p);
            choose(p + 1);
            pick.pop_back();
          }
      };
      choose(0);
    };
    rec(0);
    if (list.size() != 1) trivial = false;
    per_group.push_back(list);
  }
  {
    FoldCombos& fc = P->fc;
    fc.nletters = L;
    int total = 1;
    for (auto& l : per_group) total *= (int)l.size();
    FNO_REQUIRE(total <= kMaxCombos, kEINVAL, "antisymmetrizer too large: " + spec);
    fc.ncombo = total;
    for (int c = 0; c < total; ++c) {
      int rem = c;
      int sign = 1;
      for (int l = 0; l < kMaxLetters; ++l) fc.src[c][l] = (int8_t)(l < L ? l : 0);
      for (size_t q = 0; q < go.size(); ++q) {
        int nq = (int)per_group[q].size();
        int pick = rem % nq;
        rem /= nq;
        auto& e = per_group[q][pick];
        sign *= e.second;
        for (size_t s = 0; s < go[q].size(); ++s) fc.src[c][go[q][s]] = (int8_t)e.first[s];
      }
      fc.sign[c] = (int8_t)sign;
    }
  }

  // zero-copy decisions (FP64 only: mixed precision always converts)
  auto same = [](const std::vector<std::vector<int>>& a, const std::vector<std::vector<int>>& b) { return a == b; };
  auto cat = [](std::vector<std::vector<int>> a, const std::vector<std::vector<int>>& b) {
    a.insert(a.end(), b.begin(), b.end());
    return a;
  };
  if ((prec == Prec::FP64 || !P->B) && P->A->full_view()) {
    if (same(ga_st, cat(mg, kg))) {
      P->a_direct = true;
      P->a_kfast = true;
      P->lda = P->K.size;
    } else if (same(ga_st, cat(kg, mg))) {
      P->a_direct = true;
      P->a_kfast = false;
      P->lda = P->M.size;
    }
  }
  if (P->B && prec == Prec::FP64 && P->B->full_view()) {
    if (same(gb_st, cat(kg, ngp))) {
      P->b_direct = true;
      P->b_nfast = true;
      P->ldb = P->N.size;
    } else if (same(gb_st, cat(ngp, kg))) {
      P->b_direct = true;
      P->b_nfast = false;
      P->ldb = P->K.size;
    }
  }
  if (prec == Prec::FP64 && trivial && P->out->full_view() && P->B && same(go, cat(mg, ngp))) P->x_direct = true;
  // single operand whose gathered rows are the output elements in order: the
  // expansion accumulates straight into the output (no fold)
  if (!P->B && trivial && P->fc.ncombo == 1 && P->fc.sign[0] == 1 && P->out->full_view() && same(go, mg))
    P->copy_direct = true;
  if (!P->a_direct) {
    P->a_kfast = true;
    P->lda = P->K.size;
  }
  if (!P->b_direct) {
    P->b_nfast = true;
    P->ldb = P->N.size;
  }
  if (P->B && !P->a_direct) {
    CanonKey k = canon_key(P->A, ia, P->M, P->K, prec);
    P->a_cache = k.ok;
    P->a_key = k.key;
    P->a_keyT = k.keyT;
    P->a_sign = k.sign;
    P->a_signT = k.signT;
  }
  if (P->B && !P->b_direct) {
    CanonKey k = canon_key(P->B, ib, P->K, P->N, prec);
    P->b_cache = k.ok;
    P->b_key = k.key;
    P->b_keyT = k.keyT;
    P->b_sign = k.sign;
    P->b_signT = k.signT;
  }
  // table-driven expansion and fold
  if (!P->a_direct) P->a_tab_ok = build_expand_tab(tables, P->ad, ga_st, P->M, P->K, P->a_tab, P->bufs, stream);
  if (P->B && !P->b_direct)
    P->b_tab_ok = build_expand_tab(tables, P->bd, gb_st, P->K, P->N, P->b_tab, P->bufs, stream);
  if (!P->x_direct && P->out->full_view() && (int)go.size() <= kMaxOutGroups) {
    FoldTab& t = P->f_tab;
    t = FoldTab{};
    t.ngroups = (int)go.size();
    t.xcols = P->N.size;
    auto in_grp = [&](const DimGroup& G, const std::vector<int>& o) {
      for (int k = 0; k < G.g; ++k)
        if (!in(o, G.letter[k])) return false;
      return true;
    };
    for (size_t k = 0; k < go.size(); ++k) {
      const DimGroup& og = P->odims.grp[k];
      const auto& lst = per_group[k];
      const int ns = (int)lst.size();
      std::vector<int8_t> src((size_t)ns * kMaxLetters);
      for (int s = 0; s < ns; ++s) {
        for (int l = 0; l < kMaxLetters; ++l) src[(size_t)s * kMaxLetters + l] = (int8_t)(l < L ? l : 0);
        for (size_t sl = 0; sl < go[k].size(); ++sl) src[(size_t)s * kMaxLetters + go[k][sl]] = (int8_t)lst[s].first[sl];
      }
      unsigned xr = 0, xc = 0;
      for (int q = 0; q < P->M.ngroups; ++q)
        if (in_grp(P->M.grp[q], go[k])) xr |= 1u << q;
      for (int q = 0; q < P->N.ngroups; ++q)
        if (in_grp(P->N.grp[q], go[k])) xc |= 1u << q;
      int64_t* rowc = nullptr;
      int64_t* colc = nullptr;
      FNO_HIP(hipMalloc(&rowc, std::max<size_t>((size_t)ns * og.count * 8, 8)));
      P->bufs.push_back(rowc);
      FNO_HIP(hipMalloc(&colc, std::max<size_t>((size_t)ns * og.count * 8, 8)));
      P->bufs.push_back(colc);
      launch_fold_table(tables, og, ns, src.data(), L, P->M, P->N, xr, xc, rowc, colc, stream);
      t.count[k] = og.count;
      t.nshuf[k] = ns;
      t.rowc[k] = rowc;
      t.colc[k] = colc;
    }
    int total = 1;
    for (auto& l : per_group) total *= (int)l.size();
    t.ncombo = total;
    for (int c = 0; c < total; ++c) {
      int rem = c, sign = 1;
      for (size_t k = 0; k < go.size(); ++k) {
        int nq = (int)per_group[k].size();
        int pick = rem % nq;
        rem /= nq;
        t.combo[c][k] = (int8_t)pick;
        sign *= per_group[k][pick].second;
      }
      t.csign[c] = (int8_t)sign;
    }
    P->f_tab_ok = true;
  }
  P->prec = prec;
  plans_[key] = P;
  return P;
}

void Engine::execute(const Plan& p, double scale) {
  FNO_REQUIRE(p.prec == prec, kEINVAL, "plan precision mismatch: " + p.spec);
  const size_t esz = (prec == Prec::FP64) ? 8 : (prec == Prec::FP32 ? 4 : 2);
  const int64_t Msz = p.M.size, Nsz = p.N.size, Ksz = p.K.size;
  if (Msz == 0 || Nsz == 0 || p.odims.size == 0) return;
  const void *A = nullptr, *Alo = nullptr, *B = nullptr, *Blo = nullptr;
  if (!p.B) {
    // single operand: fold A (gathered as an M x 1 FP64 matrix) into the output
    FNO_REQUIRE(Ksz == 1, kEINVAL, "single-operand term with summation: " + p.spec);
    const void* X = p.A->d + p.A->base;
    const bool tm = timed(p.f_tab_ok ? "fno::copy (expand_tab + fold_tab)" : "fno::copy (expand + fold)") && !rec_;
    hipEvent_t e0 = tm ? event() : nullptr;
    if (e0) FNO_HIP(hipEventRecord(e0, stream));
    if (p.copy_direct && p.a_tab_ok && !p.a_direct) {
      launch_expand_tab_acc(p.a_tab, p.A->d, p.out->d, p.alpha * scale, stream);
      if (e0) {
        hipEvent_t e1 = event();
        FNO_HIP(hipEventRecord(e1, stream));
        prof_mark("fno::copy (expand_tab)", p.spec, 0, (double)Msz * 24.0, e0, e1);
      }
      return;
    }
    if (!p.a_direct) {
      void* a = workspace(0, (size_t)Msz * 8);
      if (p.a_tab_ok)
        launch_expand_tab(p.a_tab, p.A->d, a, nullptr, Prec::FP64, stream);
      else
        launch_expand(tables, p.ad, p.M, p.K, p.A->d, a, nullptr, Prec::FP64, true, stream);
      X = a;
    }
    if (p.f_tab_ok)
      launch_fold_tab(p.f_tab, X, Prec::FP64, p.out->d, p.alpha * scale, p.odims.size, stream);
    else
      launch_fold(tables, p.od, p.odims, p.M, p.N, p.fc, X, Prec::FP64, p.out->d, p.alpha * scale, stream);
    if (e0) {
      hipEvent_t e1 = event();
      FNO_HIP(hipEventRecord(e1, stream));
      prof_mark(p.f_tab_ok ? "fno::copy (expand_tab + fold_tab)" : "fno::copy (expand + fold)", p.spec, 0,
                16.0 * (double)p.odims.size, e0, e1);
    }
    return;
  }
  // operand matrices: the tensor itself, a cached expansion (direct or
  // transposed), or a fresh expansion into the cache or a workspace
  double factor = 1.0;
  bool a_kfast = p.a_kfast, b_nfast = p.b_nfast;
  int64_t lda = p.lda, ldb = p.ldb;
  // rows of a table-expanded operand start 16-byte aligned, so the GEMM can
  // use vector loads: 16-element boundaries for wide rows, 4-element ones
  // (8 for the 2-byte split-BF16 halves) for rows of 16..127; narrower rows
  // stay packed
  const int64_t mid_align = prec == Prec::BF16X3 ? 8 : 4;
  auto padded = [mid_align](bool tab_ok, int64_t cols) {
    if (!tab_ok || cols < 16) return cols;
    return cols >= 128 ? (cols + 15) / 16 * 16 : (cols + mid_align - 1) / mid_align * mid_align;
  };
  auto expand_into = [&](const Tensor* t, bool tab_ok, const ExpandTab& tab, const OperandDesc& od, const MatDim& r,
                         const MatDim& c, void* hi, void* lo, int64_t ld) {
    const bool tm = timed(tab_ok ? "fno::expand_tab" : "fno::expand_kernel") && !rec_;
    hipEvent_t e0 = tm ? event() : nullptr;
    if (e0) FNO_HIP(hipEventRecord(e0, stream));
    if (tab_ok) {
      ExpandTab tl = tab;
      tl.ld = ld;
      launch_expand_tab(tl, t->d, hi, lo, prec, stream);
    } else
      launch_expand(tables, od, r, c, t->d, hi, lo, prec, true, stream);
    if (e0) {
      hipEvent_t e1 = event();
      FNO_HIP(hipEventRecord(e1, stream));
      prof_mark(tab_ok ? "fno::expand_tab" : "fno::expand_kernel", p.spec, 0,
                (double)(r.size * c.size) * (double)(esz * (prec == Prec::BF16X3 ? 2 : 1)), e0, e1);
    }
  };
  // returns true when the operand was served from (or expanded into) the cache
  auto cached = [&](const Tensor* t, bool ok, const std::string& key, const std::string& keyT, int sgn, int sgnT,
                    int64_t rows, int64_t cols, bool tab_ok, const ExpandTab& tab, const OperandDesc& od,
                    const MatDim& r, const MatDim& c, const void*& hi, const void*& lo, bool& fast, int64_t& ld) {
    if (!ok || !is_cacheable(t->name)) return false;
    auto other_lane = [&](const CacheEntry& ce) {
      if (fork_marked_ && ce.ready_set && ce.lane != lane_) FNO_HIP(hipStreamWaitEvent(stream, ce.ready, 0));
    };
    // an entry the other lane made in the current fork cycle is not used
    // (that would make this lane wait for the other one): each lane then
    // keeps its own copy, under a lane-tagged key; entries made before the
    // fork, or in an earlier (joined) cycle, serve both lanes
    auto usable = [&](const CacheEntry& ce) {
      return ce.valid && !(fork_marked_ && ce.ready_set && ce.lane != lane_ && ce.fork_id == fork_id_);
    };
    const std::string own = lane_ ? "1|" : "0|";
    for (const std::string* k : {&key, &keyT})
      for (const std::string& kk : {*k, own + *k}) {
        auto it = ecache_.find(kk);
        if (it == ecache_.end() || !usable(it->second)) continue;
        other_lane(it->second);
        hi = it->second.hi;
        lo = it->second.lo;
        fast = k == &key;
        ld = it->second.ld;  // as the transpose: its row stride
        factor *= (k == &key ? sgn : sgnT) * it->second.sign;
        return true;
      }
    auto plain = ecache_.find(key);
    CacheEntry& ce = ecache_[(plain != ecache_.end() && plain->second.valid) ? own + key : key];
    const int64_t ldp = padded(tab_ok, cols);
    const size_t need = (size_t)(rows * ldp) * esz;
    if (ce.bytes < need) {
      FNO_REQUIRE(!rec_, kEINVAL, "expansion cache growth while recording");
      ++epoch;
      FNO_HIP(hipStreamSynchronize(stream));
      if (ce.hi) FNO_HIP(hipFree(ce.hi));
      if (ce.lo) FNO_HIP(hipFree(ce.lo));
      ce.hi = ce.lo = nullptr;
      ce.bytes = 0;
      FNO_HIP(hipMalloc(&ce.hi, std::max<size_t>(need, 256)));
      if (prec == Prec::BF16X3) FNO_HIP(hipMalloc(&ce.lo, std::max<size_t>(need, 256)));
      ce.bytes = need;
    }
    ce.tensor = t->name;
    ce.ld = ldp;
    expand_into(t, tab_ok, tab, od, r, c, ce.hi, ce.lo, ldp);
    ce.sign = sgn;
    ce.valid = true;
    ce.lane = lane_;
    ce.fork_id = fork_id_;
    ce.ready_set = fork_marked_;
    if (fork_marked_) {
      if (!ce.ready) {
        FNO_REQUIRE(!rec_, kEINVAL, "cache event created while recording");
        FNO_HIP(hipEventCreateWithFlags(&ce.ready, hipEventDisableTiming));
      }
      FNO_HIP(hipEventRecord(ce.ready, stream));
    }
    hi = ce.hi;
    lo = ce.lo;
    fast = true;
    ld = ldp;
    return true;
  };
  if (p.a_direct) {
    A = p.A->d + p.A->base;
  } else if (!cached(p.A, p.a_cache, p.a_key, p.a_keyT, p.a_sign, p.a_signT, Msz, Ksz, p.a_tab_ok, p.a_tab, p.ad,
                     p.M, p.K, A, Alo, a_kfast, lda)) {
    const int64_t ldp = padded(p.a_tab_ok, Ksz);
    void* a = workspace(0, (size_t)(Msz * ldp) * esz);
    void* alo = prec == Prec::BF16X3 ? workspace(3, (size_t)(Msz * ldp) * esz) : nullptr;
    expand_into(p.A, p.a_tab_ok, p.a_tab, p.ad, p.M, p.K, a, alo, ldp);
    A = a;
    Alo = alo;
    lda = ldp;
  }
  if (p.b_direct) {
    B = p.B->d + p.B->base;
  } else if (!cached(p.B, p.b_cache, p.b_key, p.b_keyT, p.b_sign, p.b_signT, Ksz, Nsz, p.b_tab_ok, p.b_tab, p.bd,
                     p.K, p.N, B, Blo, b_nfast, ldb)) {
    const int64_t ldp = padded(p.b_tab_ok, Nsz);
    void* b = workspace(1, (size_t)(Ksz * ldp) * esz);
    void* blo = prec == Prec::BF16X3 ? workspace(4, (size_t)(Ksz * ldp) * esz) : nullptr;
    expand_into(p.B, p.b_tab_ok, p.b_tab, p.bd, p.K, p.N, b, blo, ldp);
    B = b;
    Blo = blo;
    ldb = ldp;
  }
  if (prec == Prec::BF16X3)
    FNO_REQUIRE(Alo != nullptr && Blo != nullptr, kEINVAL, "split-BF16 GEMM needs expanded operands: " + p.spec);
  GemmArgs g{};
  g.prec = prec;
  g.M = Msz;
  g.N = Nsz;
  g.K = Ksz;
  g.A = A;
  g.A_lo = Alo;
  g.lda = lda;
  g.a_kfast = a_kfast;
  g.B = B;
  g.B_lo = Blo;
  g.ldb = ldb;
  g.b_nfast = b_nfast;
  g.tile = -1;
  bool deferred = false;  // the GEMM went to the sink (and so does the fold)
  auto timed_gemm = [&]() {
    // a full contraction to one number (energies): a deterministic dot
    // product, two small launches instead of a split-K GEMM and its reduction
    const bool a_contig = g.a_kfast || g.lda == 1;   // A is 1 x K
    const bool b_contig = !g.b_nfast || g.ldb == 1;  // B is K x 1
    if (g.M == 1 && g.N == 1 && prec == Prec::FP64 && a_contig && b_contig) {
      double* part = (double*)workspace(5, (size_t)dot_partial_blocks(g.K) * sizeof(double));
      launch_dot_acc((const double*)g.A, (const double*)g.B, g.K, part, (double*)g.C, g.alpha, g.beta, stream);
      return;
    }
    if (sink) {  // default tile and its split-K factor (the slices' partials in workspace 5)
      GemmArgs d = g;
      d.tile = -1;
      d.split = gemm_split_factor(d);
      d.ws = d.split > 1 ? workspace(5, gemm_split_bytes(d, d.split)) : nullptr;
      sink->gemms.push_back(d);
      deferred = true;
      return;
    }
    g.split = gemm_split_factor(g);
    if (g.split > 1) g.ws = workspace(5, gemm_split_bytes(g, g.split));
    if (autotune && !rec_ && g.tile < 0) {
      g.tile = tuned_tile(g);
      g.split = gemm_split_factor(g);
      if (g.split > 1) g.ws = workspace(5, gemm_split_bytes(g, g.split));
    }
    // the kernel and the GEMM's shape: launches of one instantiation on
    // different terms are timed and reported apart
    const std::string label = gemm_label(g) + " [" + std::to_string(Msz) + "x" + std::to_string(Nsz) + "x" +
                              std::to_string(Ksz) + "]";
    const double b = (double)esz * (double)(Msz * Ksz + Ksz * Nsz) * (prec == Prec::BF16X3 ? 2 : 1) +
                     (prec == Prec::FP64 ? 8.0 : 4.0) * (double)(Msz * Nsz);
    if (!timed(label)) {
      launch_gemm(g, stream);
      return;
    }
    auto run = [this, g, label, spec = p.spec, flops = p.flops, b]() {
      hipEvent_t e0 = event();
      FNO_HIP(hipEventRecord(e0, stream));
      launch_gemm(g, stream);
      hipEvent_t e1 = event();
      FNO_HIP(hipEventRecord(e1, stream));
      prof_mark(label, spec, flops, b, e0, e1);
    };
    if (rec_) {
      // timed inside the graph: event-record nodes on either side
      hipEvent_t e0 = nullptr, e1 = nullptr;
      FNO_HIP(hipEventCreate(&e0));
      if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        throw Error(kEDEVICE, "hipEventCreate failed");
      }
      rec_->timers.push_back({label, p.spec, p.flops, b, e0, e1});
      FNO_HIP(hipEventRecordWithFlags(e0, stream, hipEventRecordExternal));
      launch_gemm(g, stream);
      FNO_HIP(hipEventRecordWithFlags(e1, stream, hipEventRecordExternal));
    } else {
      run();
    }
  };
  if (p.x_direct) {
    g.C = p.out->d;
    g.ldc = Nsz;
    g.alpha = p.alpha * scale * factor;
    g.beta = 1.0;
    timed_gemm();
  } else {
    const size_t xsz = prec == Prec::FP64 ? 8 : 4;
    void* X = workspace(2, (size_t)(Msz * Nsz) * xsz);
    g.C = X;
    g.ldc = Nsz;
    g.alpha = factor;
    g.beta = 0.0;
    timed_gemm();
    const Prec xp = prec == Prec::FP64 ? Prec::FP64 : Prec::FP32;
    auto fold = [this, &p, X, xp, xsz, scale]() {
      const bool tm = timed(p.f_tab_ok ? "fno::fold_tab" : "fno::fold_kernel") && !rec_;
      hipEvent_t e0 = tm ? event() : nullptr;
      if (e0) FNO_HIP(hipEventRecord(e0, stream));
      if (p.f_tab_ok)
        launch_fold_tab(p.f_tab, X, xp, p.out->d, p.alpha * scale, p.odims.size, stream);
      else
        launch_fold(tables, p.od, p.odims, p.M, p.N, p.fc, X, xp, p.out->d, p.alpha * scale, stream);
      if (e0) {
        hipEvent_t e1 = event();
        FNO_HIP(hipEventRecord(e1, stream));
        prof_mark(p.f_tab_ok ? "fno::fold_tab" : "fno::fold_kernel", p.spec, 0,
                  (double)p.odims.size * (16.0 + (double)p.fc.ncombo * (double)xsz), e0, e1);
      }
    };
    if (deferred)
      sink->after.push_back(fold);
    else
      fold();
  }
  if (record) stats.push_back({p.spec, Msz, Nsz, Ksz, p.flops});
}

int Engine::tuned_tile(const GemmArgs& g0) {
  char key[160];
  std::snprintf(key, sizeof(key), "%d|%lld|%lld|%lld|%d%d", (int)g0.prec, (long long)g0.M, (long long)g0.N,
                (long long)g0.K, (int)g0.a_kfast, (int)g0.b_nfast);
  auto it = tuned_.find(key);
  if (it != tuned_.end()) return it->second.first;
  const size_t esz = g0.prec == Prec::FP64 ? 8 : 4;
  void* scratch = workspace(6, (size_t)(g0.M * g0.N) * esz);
  hipEvent_t a = nullptr, b = nullptr;
  FNO_HIP(hipEventCreate(&a));
  FNO_HIP(hipEventCreate(&b));
  // each tile: one warm-up launch, then the fastest of three timed launches;
  // the default tile is kept unless another is more than 3% faster
  const int ntile = gemm_num_tiles(g0.prec);
  std::vector<float> t_ms(ntile, 0.0f);
  for (int t = 0; t < ntile; ++t) {
    GemmArgs g = g0;
    g.tile = t;
    g.C = scratch;
    g.ldc = g.N;
    g.alpha = 1.0;
    g.beta = 0.0;
    g.split = gemm_split_factor(g);
    if (g.split > 1) g.ws = workspace(5, gemm_split_bytes(g, g.split));
    launch_gemm(g, stream);
    float best_rep = 0;
    for (int r = 0; r < 3; ++r) {
      FNO_HIP(hipEventRecord(a, stream));
      launch_gemm(g, stream);
      FNO_HIP(hipEventRecord(b, stream));
      FNO_HIP(hipEventSynchronize(b));
      float ms = 0;
      FNO_HIP(hipEventElapsedTime(&ms, a, b));
      if (r == 0 || ms < best_rep) best_rep = ms;
    }
    t_ms[t] = best_rep;
  }
  GemmArgs gd = g0;
  gd.tile = -1;
  const int def = gemm_default_tile(gd);
  int best = def;
  for (int t = 0; t < ntile; ++t)
    if (t_ms[t] < t_ms[best]) best = t;
  if (best != def && t_ms[best] > 0.97f * t_ms[def]) best = def;
  static const bool trace = std::getenv("FNO_TRACE") != nullptr;
  if (trace) {
    std::fprintf(stderr, "[fno] tile times %s (ms):", key);
    for (int t = 0; t < ntile; ++t) std::fprintf(stderr, " %d:%.4f", t, t_ms[t]);
    std::fprintf(stderr, " -> %d\n", best);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  GemmArgs g = g0;
  g.tile = best;
  tuned_[key] = {best, gemm_label(g)};
  return best;
}

std::string Engine::tuned_report() const {
  std::string js = "{";
  bool first = true;
  for (auto& kv : tuned_) {
    if (!first) js += ", ";
    first = false;
    js += "\"" + kv.first + "\": \"" + kv.second.second + "\"";
  }
  return js + "}";
}

void Engine::cache_operands(const std::vector<std::string>& names) {
  for (auto& kv : ecache_) kv.second.valid = false;
  cacheable_ = names;
}

size_t Engine::cache_bytes() const {
  size_t b = 0;
  for (auto& kv : ecache_) b += kv.second.bytes * (kv.second.lo ? 2 : 1);
  return b;
}

void Engine::term(const std::string& spec, double scale) {
  auto p = plan(spec);
  execute(*p, scale);
}

void Engine::terms(const char* const* specs, int n, double scale) {
  for (int i = 0; i < n; ++i) term(specs[i], scale);
}

}  // namespace fno

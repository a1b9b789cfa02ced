// Library context: problem data, device tensors and solver state.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "engine.hpp"
#include "triples_side.hpp"

namespace fno {

struct CCOptions {
  int max_iter = 100;
  double r_tol = 1e-8, e_tol = 1e-10;
  int diis_n = 8, diis_start = 3;
  Prec prec = Prec::FP64;
  int guess = 0;  // 0: zero amplitudes; 1: learned correction of the MP-style T3 guess (guess_model)
};

class Mlp;

struct EOMOptions {
  int nroots = 4, max_iter = 60, max_sub = 0;
  int block = 0;  // vectors per sigma evaluation (0 = nroots)
  double e_tol = 1e-8, r_tol = 1e-6;
  Prec prec = Prec::FP64;
  bool left = false;  // left eigenvectors: the solver applies the transposed sigma
};

struct EOMResult {
  std::vector<double> omega, res_norm;
  int iters = 0;
  bool converged = false;
  bool want_vectors = false;
  std::vector<double> vectors;  // nroots x dim Ritz vectors (unit 2-norm) when asked for
};

// Block layout of an amplitude-like vector: (holes, particles) per block.
struct Block {
  int nh, np;
  std::string name;
  int64_t size = 0, offset = 0;
};

class Context {
 public:
  explicit Context(int device);
  ~Context();

  int device;
  std::unique_ptr<Engine> eng;
  std::string err;

  // problem
  int nocc = 0, nvir = 0, nvir_full = 0;
  double e_nuc = 0;
  std::vector<double> fock_full;  // host, full space
  std::vector<double> fock;       // host, working space
  bool loaded = false, truncated = false, cc_ready = false, cc_done = false;
  double e_ref = 0, e_corr = 0, e_mp2_full = 0, e_mp2_trunc = 0;

  void load(int o, int v, const double* f, const double* g, double en);
  void truncate(double occt, int keep, int* kept, double* emp2, double* occ);
  int ccsdt(const CCOptions& opt, double* ec, double* et, int* iters, double* rn);
  // dev: the buffers are device memory, copied on the context's stream
  void cc_residual(Prec p, double* r1, double* r2, double* r3, double* ec, bool dev = false);
  size_t amp_size(int block) const;
  void get_amps(int block, double* buf, size_t len, bool dev = false);
  void set_amps(int block, const double* buf, size_t len, bool dev = false);

  // EOM
  size_t eom_size(int kind);
  void eom_sigma(int kind, Prec p, const double* r, double* sigma, size_t len, bool dev = false, bool left = false);
  int eom(int kind, const EOMOptions& opt, EOMResult& res);
  // resumable Davidson (used by eom() and by batched solves over several contexts)
  struct Davidson;
  Davidson* dav_begin(int kind, const EOMOptions& opt);
  void dav_sigma(Davidson& d);    // issue the pending sigma vectors (no host wait)
  bool dav_update(Davidson& d);   // one iteration's host work; true when finished
  int dav_end(EOMResult& res);    // results, releases the solver; status kOK / kENOCONV
  void dav_release();
  // Grouped sigma rounds over several contexts (fno_batch_eom_grouped): the
  // pending Davidson vectors of every instance, one block per instance and
  // round, term by term: every instance's expansions, then one grouped GEMM
  // launch per kernel instantiation over all of them (a device work queue of
  // (instance, term, tile) items, the roots of a block inside each GEMM), then
  // every instance's fold; all on the batch's stream `gs`.
  struct GroupedBuffers {
    void *pin = nullptr, *dev = nullptr, *queue = nullptr;  // item tables (pinned host, device), queue counters
    size_t items = 0;                                      // capacity of each table, in items
    hipStream_t stream = nullptr;                          // the batch stream (destroyed with the buffers)
    // fork/join events (batch stream, one per instance)
    hipEvent_t ev_s = nullptr;
    std::vector<hipEvent_t> ev;
    // the recorded sigma sweep of a round (one hipGraph over every active
    // instance) and the round structure it is valid for: active instances,
    // their engines' epochs and precisions; `seen` holds the structure of the
    // last round run from the host
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> key, seen;
    int replays = 0, recordings = 0;
    void reserve(size_t n);
    void drop_graph();
    ~GroupedBuffers();
  };
  static void dav_sigma_grouped(const std::vector<Context*>& cs, const std::vector<Davidson*>& ds,
                                GroupedBuffers& gb);

  double last_triples_flops = 0, last_all_flops = 0;
  std::vector<double> trace_e, trace_r;  // per-iteration E_corr and |r| of the last fno_ccsdt

  // learned guess: the network used when CCOptions::guess == 1 (not owned)
  Mlp* guess_model = nullptr;
  bool last_guess_accepted = false;
  // append training samples (features of every selected T3 element and the
  // targets from the converged amplitudes) to the network's data set
  void ml_collect(Mlp& m, int64_t max_samples);

  // launch mode: replay the residual sweep from a recorded hipGraph program
  bool use_graphs = true;
  // ground-state triples residual through the fused per-triple kernel
  // (triples.hpp); off: one expand / GEMM / fold sequence per term
  bool fused_r3 = true;
  hipStream_t user_stream = nullptr;  // caller's stream (fno_set_stream), kept across engine rebuilds
  bool autotune = false;              // GEMM tile autotuner (fno_set_autotune), kept across engine rebuilds
  void set_stream(hipStream_t s);
  void reset_engine(std::unique_ptr<Engine> e);
  struct EomSpace;  // per-variant layout and tensors (eom_space.hpp)
  int debug_gemm(Prec p, int tile, int64_t M, int64_t N, int64_t K, bool a_kfast, bool b_nfast, double alpha,
                 double beta, const double* A, const double* B, double* Cm);

 private:
  // working-space setup
  void setup_cc();
  void dress();
  double energy();
  void energy_terms();
  // energy terms and the copy of E into host_pin_[0], followed by e_ready_
  void energy_async();
  double* pinned();  // host_pin_ (kPinned doubles of pinned host memory), allocated on first use
  static constexpr int kPinned = 64;
  double* host_pin_ = nullptr;
  hipEvent_t e_ready_ = nullptr;
  // defer_timers: a replayed sweep's in-graph timers are read later
  void residual(bool defer_timers = false);
  void residual_body(Prec tri);
  bool fused_r3_ok() const;
  void r3_fused(Prec tri, bool t3v_ready);
  void dress_gemm_slots(double* gd, const double* t1);
  void dress_last_slot(double* gd, const double* t1);
  double* r3_y_ = nullptr;      // per-triple products Y_t (FP64-sized; FP32 modes use half)
  double* r3_c_ = nullptr;      // occupied-only operator, C(o,3) x C(o,3)
  double* r3_aring_ = nullptr;  // W3_ovvo rearranged for the ring segments
  double* r3_t3v_ = nullptr;    // T3 with one virtual letter unpacked (FP64-sized)
  double* r3_wt_ = nullptr;     // W3_vvvv transposed (FP64-sized)
  double* r3_fvvp_ = nullptr;   // F3_vv padded
  std::vector<GemmStats> r3_stats_;  // packed-GEMM flops of the replaced terms
  // T3 terms of the intermediates and of R1 / R2 from the FP64 T3v
  // (triples_side.hpp), FP64 whatever the precision of the triples products
  bool side_ok(Prec tri) const;
  void side_products();
  void side_r12();
  SideShape side_sh_{};
  double* side_buf_ = nullptr;
  std::vector<GemmStats> side_stats_;
  void plain_guess();
  double t3_rms(const double* x);
  void learned_t3(const double* x, double sx, double* t3, double* den3);
  Program cc_prog_;              // recorded residual sweep
  // the last host-launched sweep allocated nothing; the settings it ran with
  bool cc_stable_ = false;
  uint64_t cc_stable_epoch_ = 0;
  int cc_stable_prec_ = -1;
  bool cc_stable_profiled_ = false;
  std::string cc_stable_filter_;
  void tally_flops();
  double dot(const double* x, const double* y, int64_t n);

  SpaceSizes sz_;
  std::vector<Block> tblocks_;
  int64_t nt_ = 0;               // packed amplitude vector length
  double* amp_ = nullptr;        // [T1|T2|T3]
  double* res_ = nullptr;        // [R1|R2|R3]
  double* den_ = nullptr;        // denominators
  double* scratch_ = nullptr;    // dot partials
  double* dscal_ = nullptr;      // device scalars
  std::vector<double*> owned_;

  // EOM state
  std::unique_ptr<EomSpace> eom_;
  std::unique_ptr<Davidson> dav_;
  void setup_eom(int kind, int nb);
  void release_eom();

  double* alloc(int64_t n);
};

}  // namespace fno

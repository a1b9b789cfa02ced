// Ground-state CCSDT on the device: T1 dressing, residual terms, Jacobi + DIIS.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "context.hpp"
#include "triples.hpp"
#include "mlp.hpp"
#include "linalg.hpp"

namespace fno {

#include "ccsdt_terms.inc"

namespace {
template <size_t N>
int count(const char* const (&)[N]) {
  return (int)N;
}

// "name : spec" -> (name, spec)
std::pair<std::string, std::string> split_decl(const char* d) {
  std::string s(d);
  size_t c = s.find(':');
  auto trim = [](std::string x) {
    size_t a = x.find_first_not_of(' '), b = x.find_last_not_of(' ');
    return a == std::string::npos ? std::string() : x.substr(a, b - a + 1);
  };
  return {trim(s.substr(0, c)), trim(s.substr(c + 1))};
}
}  // namespace

double* Context::alloc(int64_t n) {
  double* p = nullptr;
  FNO_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(n, 1) * sizeof(double)));
  launch_fill(p, 0.0, n, eng->stream);
  owned_.push_back(p);
  return p;
}

double Context::dot(const double* x, const double* y, int64_t n) {
  launch_dots(x, 0, 1, y, n, scratch_, dscal_, eng->stream);
  double r;
  FNO_HIP(hipMemcpyAsync(&r, dscal_, sizeof(double), hipMemcpyDeviceToHost, eng->stream));
  FNO_HIP(hipStreamSynchronize(eng->stream));
  return r;
}

// Views "name = parent(s0,s1,...)" with s = o (occupied), v (virtual), n (all).
static void make_views(Engine& e, const char* const* views, int nviews, int nocc, int nvir) {
  for (int i = 0; i < nviews; ++i) {
    std::string s(views[i]);
    size_t eq = s.find('='), lp = s.find('('), rp = s.find(')');
    std::string name = s.substr(0, eq);
    name.erase(std::remove(name.begin(), name.end(), ' '), name.end());
    std::string par = s.substr(eq + 1, lp - eq - 1);
    par.erase(std::remove(par.begin(), par.end(), ' '), par.end());
    std::vector<std::pair<int, int>> rng;
    for (char c : s.substr(lp + 1, rp - lp - 1)) {
      if (c == 'o') rng.push_back({0, nocc});
      if (c == 'v') rng.push_back({nocc, nvir});
      if (c == 'n') rng.push_back({0, nocc + nvir});
    }
    e.view(name, e.get(par), rng);
  }
}

void Context::setup_cc() {
  Engine& e = *eng;
  const int o = nocc, v = nvir, n = nocc + nvir;
  sz_.n = {{'o', o}, {'v', v}, {'n', n}};
  // contiguous amplitude / residual vectors [1|2|3]
  tblocks_ = {{1, 1, "1"}, {2, 2, "2"}, {3, 3, "3"}};
  const char* specs[3] = {"o,v", "oo,vv", "ooo,vvv"};
  nt_ = 0;
  for (int k = 0; k < 3; ++k) {
    tblocks_[k].size = Engine::spec_size(specs[k], sz_);
    tblocks_[k].offset = nt_;
    nt_ += tblocks_[k].size;
  }
  amp_ = alloc(nt_);
  res_ = alloc(nt_);
  den_ = alloc(nt_);
  scratch_ = alloc(256 * 1024);  // per-block partial sums of dot products and of the DIIS step
  dscal_ = alloc(1024);
  for (int k = 0; k < 3; ++k) {
    e.create("T" + tblocks_[k].name, specs[k], sz_, amp_ + tblocks_[k].offset);
    e.create("R" + tblocks_[k].name, specs[k], sz_, res_ + tblocks_[k].offset);
    e.create("D" + tblocks_[k].name, specs[k], sz_, den_ + tblocks_[k].offset);
  }
  for (int i = 0; i < count(kCCDecl); ++i) {
    auto d = split_decl(kCCDecl[i]);
    if (e.has(d.first)) continue;
    e.create(d.first, d.second, sz_);
  }
  // dense integrals of the working space and dressing work arrays
  Tensor* G = e.get("G");
  e.set_sym(G, {{0, 1}, {2, 3}});
  Tensor* Gd = e.create("Gd", "n,n,n,n", sz_);
  e.set_sym(Gd, {{0, 1}, {2, 3}});
  for (const char* nm : {"Fd", "Xt", "Yt", "Ftmp", "Ident"}) e.create(nm, "n,n", sz_);
  e.create("Iocc", "o,o", sz_);
  {
    std::vector<double> I((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) I[(size_t)i * n + i] = 1.0;
    FNO_HIP(hipMemcpy(e.get("Ident")->d, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<double> Io((size_t)o * o, 0.0);
    for (int i = 0; i < o; ++i) Io[(size_t)i * o + i] = 1.0;
    FNO_HIP(hipMemcpy(e.get("Iocc")->d, Io.data(), Io.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  make_views(e, kCCViews, count(kCCViews), o, v);
  // fused triples residual: its buffers, and the packed-GEMM flops of the
  // terms it replaces (the algorithmic count both paths report)
  if (o >= 3 && v >= 3 && v <= 64) {
    r3_y_ = alloc(r3_fused_y_elems(o, v));
    r3_c_ = alloc((int64_t)binom_host(o, 3) * (int64_t)binom_host(o, 3));
    r3_aring_ = alloc(r3_ring_operand_elems(o, v));
    r3_t3v_ = alloc(r3_fused_t3v_elems(o, v));
    r3_wt_ = alloc(r3_fused_wt_elems(v));
    r3_fvvp_ = alloc(r3_fvv_padded_elems(v));
  }
  e.view("Xt_vo", e.get("Xt"), {{o, v}, {0, o}});
  e.view("Yt_vo", e.get("Yt"), {{o, v}, {0, o}});
  e.view("Gd_nono", Gd, {{0, n}, {0, o}, {0, n}, {0, o}});
  // denominators D = sum f_holes - sum f_particles over the packed blocks
  std::vector<double> eo(o), ev(v);
  for (int i = 0; i < o; ++i) eo[i] = fock[(size_t)i * n + i];
  for (int a = 0; a < v; ++a) ev[a] = fock[(size_t)(o + a) * n + (o + a)];
  double* d_eo = alloc(o);
  double* d_ev = alloc(v);
  FNO_HIP(hipMemcpy(d_eo, eo.data(), o * sizeof(double), hipMemcpyHostToDevice));
  FNO_HIP(hipMemcpy(d_ev, ev.data(), v * sizeof(double), hipMemcpyHostToDevice));
  for (int k = 0; k < 3; ++k) {
    MatDim md{};
    int nh = tblocks_[k].nh, np = tblocks_[k].np;
    md.ngroups = 2;
    md.grp[0].g = nh;
    md.grp[0].n = o;
    md.grp[0].count = (int64_t)binom_host(o, nh);
    md.grp[1].g = np;
    md.grp[1].n = v;
    md.grp[1].count = (int64_t)binom_host(v, np);
    for (int s = 0; s < nh; ++s) md.grp[0].letter[s] = (int8_t)s;
    for (int s = 0; s < np; ++s) md.grp[1].letter[s] = (int8_t)(nh + s);
    md.size = md.grp[0].count * md.grp[1].count;
    launch_denominators(e.tables, md, nh, d_eo, d_ev, den_ + tblocks_[k].offset, e.stream);
  }
  r3_stats_.clear();
  side_stats_.clear();
  if (r3_y_) {
    const Prec keep = e.prec;
    e.prec = Prec::FP64;
    for (const char* t : kCCR3) r3_stats_.push_back(e.term_shape(t));
    side_sh_ = side_shape(o, v);
    side_buf_ = alloc(side_sh_.total);
    for (const char* t : kCCInter3)
      if (std::strstr(t, "T3[")) side_stats_.push_back(e.term_shape(t));
    for (const char* t : kCCR1)
      if (std::strstr(t, "T3[")) side_stats_.push_back(e.term_shape(t));
    for (const char* t : kCCR2)
      if (std::strstr(t, "T3[")) side_stats_.push_back(e.term_shape(t));
    e.prec = keep;
  }
  cc_ready = true;
}

// H^ = e^{-T1} H e^{T1}: creation indices transform with X = 1 - t1 (block
// X[a,i] = -t_i^a), annihilation indices with Y = 1 + t1 (Y[a,i] = t_i^a).
// Each of the four index transformations is one GEMM that rotates the
// contracted index to the back, so all operands are used in place.
// All four slots on Gd (already a copy of G): slots 0 and 3 as GEMMs, 1 and
// 2 as strided passes.
void Context::dress_gemm_slots(double* gd, const double* t1) {
  Engine& e = *eng;
  const int n = nocc + nvir;
  const int64_t n3 = (int64_t)n * n * n;
  // slot 0 is a plain GEMM: Gd[a, :] -= sum_i t1[i][a] Gd[i, :]  (v x n^3, K = o)
  GemmArgs s0{};
  s0.prec = Prec::FP64;
  s0.M = nvir;
  s0.N = n3;
  s0.K = nocc;
  s0.A = t1;
  s0.lda = nvir;
  s0.a_kfast = false;
  s0.B = gd;
  s0.ldb = n3;
  s0.b_nfast = true;
  s0.C = gd + (int64_t)nocc * n3;
  s0.ldc = n3;
  s0.alpha = -1.0;
  s0.beta = 1.0;
  s0.tile = -1;
  s0.split = 1;
  launch_gemm(s0, e.stream);
  // slots 1 and 2: strided slices, one thread per position of the other slots
  launch_dress_pass(gd, t1, nocc, nvir, 1, true, e.stream);
  launch_dress_pass(gd, t1, nocc, nvir, 2, false, e.stream);
  dress_last_slot(gd, t1);
}

// slot 3: a plain GEMM on the rows of Gd: Gd[:, i] += sum_a Gd[:, a] t1[i][a]  (n^3 x o, K = v)
void Context::dress_last_slot(double* gd, const double* t1) {
  Engine& e = *eng;
  const int n = nocc + nvir;
  const int64_t n3 = (int64_t)n * n * n;
  GemmArgs s3{};
  s3.prec = Prec::FP64;
  s3.M = n3;
  s3.N = nocc;
  s3.K = nvir;
  s3.A = gd + nocc;
  s3.lda = n;
  s3.a_kfast = true;
  s3.B = t1;
  s3.ldb = nvir;
  s3.b_nfast = false;
  s3.C = gd;
  s3.ldc = n;
  s3.alpha = 1.0;
  s3.beta = 1.0;
  s3.tile = -1;
  s3.split = 1;
  launch_gemm(s3, e.stream);
}

void Context::dress() {
  Engine& e = *eng;
  const int n = nocc + nvir;
  const int64_t nn = (int64_t)n * n;
  launch_axpby(e.get("Xt")->d, e.get("Ident")->d, 1.0, 0.0, nn, e.stream);
  launch_axpby(e.get("Yt")->d, e.get("Ident")->d, 1.0, 0.0, nn, e.stream);
  e.term("Xt_vo[am] -= 1 * T1[ma]");
  e.term("Yt_vo[am] += 1 * T1[ma]");
  // g^[PQRS] = sum X[P,p] X[Q,q] g[pqrs] Y[r,R] Y[s,S]: X and Y differ from
  // the identity only in their virtual-occupied block, so each slot is an
  // in-place update of one slice (K = o for X, K = v for Y)
  Tensor* gd = e.get("Gd");
  Tensor* g0 = e.get("G");
  const double* t1 = e.get("T1")->d;  // t1[i][a], o x v
  if (launch_dress_first_slot(g0->d, gd->d, t1, nocc, nvir, e.stream)) {
    // slot 0 done with the copy; slots 1 and 2 are strided passes (one
    // thread per position of the other slots), slot 3 a GEMM on the rows
    launch_dress_pass(gd->d, t1, nocc, nvir, 1, true, e.stream);
    launch_dress_pass(gd->d, t1, nocc, nvir, 2, false, e.stream);
    dress_last_slot(gd->d, t1);
  } else {
    FNO_HIP(hipMemcpyAsync(gd->d, g0->d, (size_t)g0->elems * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    dress_gemm_slots(gd->d, t1);
  }
  // f^ = X h Y + sum_i g^[p i q i]
  e.zero(e.get("Ftmp"));
  e.zero(e.get("Fd"));
  e.term("Ftmp[pQ] += 1 * Hcore[pq] * Yt[qQ]");
  e.term("Fd[PQ] += 1 * Xt[Pp] * Ftmp[pQ]");
  e.term("Fd[pq] += 1 * Gd_nono[piqj] * Iocc[ij]");
}

double* Context::pinned() {
  if (!host_pin_) FNO_HIP(hipHostMalloc((void**)&host_pin_, kPinned * sizeof(double), hipHostMallocDefault));
  return host_pin_;
}

// E[0] = the correlation energy of the current amplitudes, one closed-form
// pass (the terms of kCCEnergy folded onto unique index pairs)
void Context::energy_terms() {
  Engine& e = *eng;
  launch_cc_energy(e.get("F0")->d, e.get("G")->d, amp_ + tblocks_[0].offset, amp_ + tblocks_[1].offset, nocc, nvir,
                   scratch_, e.get("E")->d, e.stream);
}

void Context::energy_async() {
  Engine& e = *eng;
  energy_terms();
  FNO_HIP(hipMemcpyAsync(pinned(), e.get("E")->d, sizeof(double), hipMemcpyDeviceToHost, e.stream));
  if (!e_ready_) FNO_HIP(hipEventCreateWithFlags(&e_ready_, hipEventDisableTiming));
  FNO_HIP(hipEventRecord(e_ready_, e.stream));
}

double Context::energy() {
  Engine& e = *eng;
  energy_terms();
  double r;
  FNO_HIP(hipMemcpyAsync(&r, e.get("E")->d, sizeof(double), hipMemcpyDeviceToHost, e.stream));
  FNO_HIP(hipStreamSynchronize(e.stream));
  return r;
}

// The residual sweep is the same sequence of launches every iteration: once
// an eager sweep has run without allocating anything, the next one is
// recorded into hipGraph segments and later sweeps replay them (host launch
// overhead removed).  Any allocation in the engine invalidates the recording.
void Context::residual(bool defer_timers) {
  Engine& e = *eng;
  const Prec tri = e.prec;  // precision of the triples-residual contractions
  auto matches = [&]() {
    return cc_prog_.valid() && cc_prog_.epoch == e.epoch && cc_prog_.prec == (int)tri &&
           cc_prog_.profiled == e.profile && cc_prog_.filter == e.profile_filter;
  };
  if (use_graphs && matches()) {
    e.replay(cc_prog_, defer_timers);
    e.prec = tri;
    return;
  }
  e.flush_timers(cc_prog_);
  cc_prog_.clear();
  if (use_graphs && cc_stable_ && cc_stable_epoch_ == e.epoch && cc_stable_prec_ == (int)tri &&
      cc_stable_profiled_ == e.profile && cc_stable_filter_ == e.profile_filter) {
    bool recorded = false;
    e.begin_record(cc_prog_);
    try {
      residual_body(tri);
      e.end_record(cc_prog_);
      recorded = true;
    } catch (const Error&) {
      // something in the sweep cannot be recorded (it needed memory or a
      // host synchronization): discard the capture and launch from the host
      e.abort_record();
      e.prec = tri;
      cc_stable_ = false;
    }
    if (recorded && cc_prog_.valid()) {
      e.replay(cc_prog_, defer_timers);
      return;
    }
  }
  const uint64_t before = e.epoch;
  residual_body(tri);
  cc_stable_ = e.epoch == before;
  cc_stable_epoch_ = e.epoch;
  cc_stable_prec_ = (int)tri;
  cc_stable_profiled_ = e.profile;
  cc_stable_filter_ = e.profile_filter;
}

void Context::residual_body(Prec tri) {
  Engine& e = *eng;
  e.prec = Prec::FP64;
  std::vector<Tensor*> cleared;
  for (const char* nm : {"F2_vv", "F2_oo", "W2_oooo", "W2_vvvv", "W2_ovvo", "F3_vv", "F3_oo", "W3_oooo", "W3_vvvv",
                         "W3_ovvo", "W3_vvvo", "W3_ovoo"})
    cleared.push_back(e.get(nm));
  e.zero_many(cleared, res_, nt_);
  dress();
  e.stats.clear();
  e.record = true;
  {
    // the amplitudes are fixed during the sweep: their expanded operand
    // matrices are shared between terms (the ring, R1 and the F_ov term of R2
    // use one layout of T3; the T3 pieces of W3_vvvo/W3_ovoo and the G terms
    // of R2 another).  The triples terms are issued first so that the largest
    // GEMM (the ring) fixes the stored orientation.
    CacheScope cache(e, {"T1", "T2", "T3"});
    struct Join {  // the side lane is joined on every exit
      Engine& e;
      ~Join() {
        try {
          e.join_side();
        } catch (...) {
        }
      }
    } join{e};
    // two lanes from here: the triples intermediates (split over both lanes
    // where T3 is not involved) and residual on the main stream; the doubles
    // intermediates and the T2 parts of the singles and doubles residual on
    // the side lane, concurrently (they read T1, T2 and the dressed integrals,
    // and write R1, R2 and the W2/F2 blocks).  The T3
    // feedback into R1 and R2 follows the triples on the main stream: it uses
    // expansions of T3 made by the triples terms, and the side lane has
    // finished long before the last triples term (the ring), which therefore
    // runs alone.  Dressing, intermediates and the singles/doubles residual
    // are FP64; the triples residual contractions run in the requested
    // precision and accumulate into the FP64 residual.
    e.fork_mark();
    const bool side = side_ok(tri);
    if (side) {
      // the intermediates without T3 over both lanes, each output block's
      // terms on one lane (W3_vvvv, W3_ovvo and F3 on the side lane, W3_oooo,
      // W3_vvvo and W3_ovoo here), joined before the T3 pieces of W3_vvvo /
      // W3_ovoo from T3v; the doubles lane then forks again
      auto side_block = [](const char* t) {
        return !std::strncmp(t, "W3_vvvv", 7) || !std::strncmp(t, "W3_ovvo", 7) || !std::strncmp(t, "F3_", 3);
      };
      e.begin_side();
      for (const char* t : kCCInter3)
        if (!std::strstr(t, "T3[") && side_block(t)) e.term(t);
      e.end_side();
      for (const char* t : kCCInter3)
        if (!std::strstr(t, "T3[") && !side_block(t)) e.term(t);
      e.join_side();
      e.fork_mark();
      side_products();
    } else {
      e.terms(kCCInter3, count(kCCInter3));
    }
    e.prec = tri;
    if (fused_r3_ok())
      r3_fused(tri, side && tri == Prec::FP64);
    else
      e.terms(kCCR3, count(kCCR3));
    e.prec = Prec::FP64;
    std::vector<const char*> late;
    e.begin_side();
    e.terms(kCCInter2, count(kCCInter2));
    for (const char* t : kCCR1) (std::strstr(t, "T3[") ? late.push_back(t) : e.term(t));
    for (const char* t : kCCR2) (std::strstr(t, "T3[") ? late.push_back(t) : e.term(t));
    e.end_side();
    e.join_side();
    if (side)
      side_r12();
    else
      for (const char* t : late) e.term(t);
  }
  e.prec = tri;
  e.record = false;
  tally_flops();
}

// The side products read an FP64 T3v and finish before the fused kernel, so
// every precision can use them: with FP32 products the fused kernel then
// rebuilds the same buffer in FP32.
bool Context::side_ok(Prec) const { return side_buf_ != nullptr && fused_r3_ok(); }

// T3v (FP64) first, then the integral rows, the NT / NN products and the
// W3_vvvo / W3_ovoo T3 pieces (triples_side.hpp); the R1 / R2 gathers wait for
// the side lane (side_r12).  The packed-GEMM flops of the replaced terms are
// recorded as the per-term path would record them.
void Context::side_products() {
  Engine& e = *eng;
  const int o = nocc, v = nvir;
  const SideShape& sh = side_sh_;
  double* T3 = amp_ + tblocks_[2].offset;
  e.timed_launch("fno::r3_t3v_kernel", "T3v", 0,
                 8.0 * (double)tblocks_[2].size + 8.0 * (double)r3_fused_t3v_elems(o, v),
                 [&]() { launch_r3_t3v(e.tables, o, v, T3, r3_t3v_, Prec::FP64, e.stream); });
  e.timed_launch("fno::side_slab_kernel + side_a2_kernel", "side T3 terms: integral rows", 0,
                 8.0 * (double)(sh.a2 + (int64_t)sh.nt * sh.mt2 * 64 * sh.ep),
                 [&]() { launch_side_operands(e.tables, sh, e.get("Gd")->d, e.get("Fd")->d, side_buf_, e.stream); });
  double fl = 0;
  for (auto& st : side_stats_) fl += st.flops;
  e.timed_launch("fno::side_nt_kernel + side_nn_kernel", "side T3 terms: products", fl,
                 8.0 * (double)(r3_fused_y_elems(o, v) + sh.o2 - sh.s + (sh.total - sh.o2)),
                 [&]() { launch_side_products(e.tables, sh, (const double*)r3_t3v_, side_buf_, e.stream); });
  e.timed_launch("fno::side_w3_kernel", "side T3 terms: W3_vvvo, W3_ovoo", 0,
                 8.0 * (double)(sh.total - sh.wp) + 16.0 * o * v * (sh.nv2 + sh.no2),
                 [&]() { launch_side_w3(e.tables, sh, side_buf_, e.get("W3_vvvo")->d, e.get("W3_ovoo")->d,
                                        e.stream); });
  if (e.record)
    for (auto& st : side_stats_) e.stats.push_back(st);
}

void Context::side_r12() {
  Engine& e = *eng;
  const SideShape& sh = side_sh_;
  e.timed_launch("fno::side_r12_kernel", "side T3 terms: R1, R2", 0,
                 8.0 * (double)(sh.wp - sh.o2) + 16.0 * ((double)sh.no2 * sh.nv2 + nocc * nvir),
                 [&]() {
                   launch_side_r12(e.tables, sh, side_buf_, res_ + tblocks_[0].offset, res_ + tblocks_[1].offset,
                                   e.stream);
                 });
}

bool Context::fused_r3_ok() const {
  return fused_r3 && nocc >= 3 && nvir >= 3 && nvir <= 64 && nocc <= eng->tables.dec_max_n[3] && r3_y_ != nullptr;
}

// The triples residual of kCCR3 in one pass (triples.hpp): the occupied-only
// operator C from W3_oooo and F3_oo, the per-triple products Y_t of every
// other term in one fused GEMM, the P(a/bc) fold of Y into R3, and
// R3 += C T3.  The packed-GEMM flops of the replaced terms are recorded as
// the per-term path would record them.
void Context::r3_fused(Prec tri, bool t3v_ready) {
  Engine& e = *eng;
  const int o = nocc, v = nvir;
  const int nt = (int)binom_host(o, 3), nv3 = (int)binom_host(v, 3);
  double* T3 = amp_ + tblocks_[2].offset;
  double* R3 = res_ + tblocks_[2].offset;
  const double bytes_t3 = 8.0 * (double)tblocks_[2].size;
  const double esz = tri == Prec::FP64 ? 8.0 : 4.0;
  if (!t3v_ready)
    e.timed_launch("fno::r3_t3v_kernel", "R3 fused: T3v", 0, bytes_t3 + esz * (double)r3_fused_t3v_elems(o, v),
                   [&]() { launch_r3_t3v(e.tables, o, v, T3, r3_t3v_, tri, e.stream); });
  e.timed_launch("fno::r3_wt_kernel", "R3 fused: W3_vvvv^T", 0, (8.0 + esz) * (double)r3_fused_wt_elems(v),
                 [&]() { launch_r3_wt(v, e.get("W3_vvvv")->d, r3_wt_, tri, e.stream); });
  e.timed_launch("fno::r3_ring_operand_kernel", "R3 fused: W3_ovvo rearranged", 0, 16.0 * o * v * o * v,
                 [&]() {
                   launch_r3_ring_operand(e.get("W3_ovvo")->d, e.get("F3_vv")->d, o, v, r3_aring_, r3_fvvp_,
                                          e.stream);
                 });
  e.timed_launch("fno::r3_occ_operator_kernel", "R3 fused: occupied operator", 0, 8.0 * nt * nt,
                 [&]() { launch_r3_occ_operator(e.tables, o, e.get("W3_oooo")->d, e.get("F3_oo")->d, r3_c_,
                                                e.stream); });
  R3FusedArgs a;
  a.o = o;
  a.v = v;
  a.T3 = T3;
  a.T3v = r3_t3v_;
  a.WT = r3_wt_;
  a.T2 = amp_ + tblocks_[1].offset;
  a.Wvvvv = e.get("W3_vvvv")->d;
  a.Fvvp = r3_fvvp_;
  a.Aring = r3_aring_;
  a.Wvvvo = e.get("W3_vvvo")->d;
  a.Wovoo = e.get("W3_ovoo")->d;
  a.Y = r3_y_;
  a.ldy = r3_fused_ldy(v);
  double fl = 0;
  for (auto& st : r3_stats_)
    if (st.term.find("W3_oooo") == std::string::npos && st.term.find("F3_oo") == std::string::npos) fl += st.flops;
  const double ybytes = (tri == Prec::FP64 ? 8.0 : 4.0) * (double)r3_fused_y_elems(o, v);
  // algorithmic bytes: T3v read and Y written once, W3_vvvv^T (C(v,2) rows),
  // the ring operand, W3_vvvo, W3_ovoo and T2 read once
  const double no2 = (double)binom_host(o, 2), nv2 = (double)binom_host(v, 2);
  const double fused_bytes = 2.0 * ybytes + esz * nv2 * (double)a.ldy +
                             8.0 * ((double)r3_ring_operand_elems(o, v) + o * v * nv2 + o * v * no2 + no2 * nv2);
  e.timed_launch(tri == Prec::FP64   ? "fno::r3_fused_kernel<double>"
                 : tri == Prec::FP32 ? "fno::r3_fused_kernel<float>"
                                     : "fno::r3_fused_kernel<float, true>",
                 "R3 fused: pp-ladder, ring, drivers, one-body vv", fl, fused_bytes,
                 [&]() { launch_r3_fused(e.tables, a, tri, e.stream); });
  e.timed_launch("fno::r3_fold_kernel", "R3 fused: P(a/bc) fold", 0, 3.0 * ybytes / v + 2.0 * bytes_t3,
                 [&]() { launch_r3_fold(e.tables, o, v, r3_y_, a.ldy, tri, R3, e.stream); });
  // R3 += C T3 (FP64: a small GEMM on the packed rows)
  GemmArgs g{};
  g.prec = Prec::FP64;
  g.M = nt;
  g.N = nv3;
  g.K = nt;
  g.A = r3_c_;
  g.lda = nt;
  g.a_kfast = true;
  g.B = T3;
  g.ldb = nv3;
  g.b_nfast = true;
  g.C = R3;
  g.ldc = nv3;
  g.alpha = 1.0;
  g.beta = 1.0;
  g.tile = -1;
  g.split = 1;
  double flo = 0;
  for (auto& st : r3_stats_)
    if (st.term.find("W3_oooo") != std::string::npos || st.term.find("F3_oo") != std::string::npos) flo += st.flops;
  e.timed_launch(gemm_label(g) + " [R3 += C T3]", "R3 fused: hh-ladder, F_oo", flo, 3.0 * bytes_t3,
                 [&]() { launch_gemm(g, e.stream); });
  if (e.record)
    for (auto& st : r3_stats_) e.stats.push_back(st);
}

void Context::tally_flops() {
  double tri = 0, all = 0;
  for (auto& s : eng->stats) {
    all += s.flops;
    if (s.term.find("T3[") != std::string::npos || s.term.find("R3[") != std::string::npos) tri += s.flops;
  }
  last_triples_flops = tri;
  last_all_flops = all;
}

size_t Context::amp_size(int block) const {
  if (!cc_ready || block < 1 || block > 3) return 0;
  return (size_t)tblocks_[block - 1].size;
}

void Context::get_amps(int block, double* buf, size_t len, bool dev) {
  FNO_REQUIRE(cc_ready, kESTATE, "no amplitudes: call fno_ccsdt or fno_set_amplitudes first");
  FNO_REQUIRE(block >= 1 && block <= 3 && len == amp_size(block), kEINVAL, "bad amplitude block or length");
  if (dev) {
    FNO_HIP(hipMemcpyAsync(buf, amp_ + tblocks_[block - 1].offset, len * sizeof(double), hipMemcpyDeviceToDevice,
                           eng->stream));
    return;
  }
  FNO_HIP(hipMemcpyAsync(buf, amp_ + tblocks_[block - 1].offset, len * sizeof(double), hipMemcpyDeviceToHost,
                         eng->stream));
  FNO_HIP(hipStreamSynchronize(eng->stream));
}

void Context::set_amps(int block, const double* buf, size_t len, bool dev) {
  FNO_REQUIRE(loaded, kESTATE, "no Hamiltonian loaded");
  if (!cc_ready) setup_cc();
  FNO_REQUIRE(block >= 1 && block <= 3 && len == amp_size(block), kEINVAL, "bad amplitude block or length");
  if (dev) {
    FNO_HIP(hipMemcpyAsync(amp_ + tblocks_[block - 1].offset, buf, len * sizeof(double), hipMemcpyDeviceToDevice,
                           eng->stream));
    return;
  }
  for (size_t i = 0; i < len; ++i) FNO_REQUIRE(std::isfinite(buf[i]), kENONFINITE, "non-finite amplitude");
  FNO_HIP(hipMemcpyAsync(amp_ + tblocks_[block - 1].offset, buf, len * sizeof(double), hipMemcpyHostToDevice,
                         eng->stream));
  FNO_HIP(hipStreamSynchronize(eng->stream));
}

void Context::cc_residual(Prec p, double* r1, double* r2, double* r3, double* ec, bool dev) {
  FNO_REQUIRE(loaded, kESTATE, "no Hamiltonian loaded");
  if (!cc_ready) setup_cc();
  eng->prec = p;
  residual();
  eng->prec = Prec::FP64;
  double* outs[3] = {r1, r2, r3};
  for (int k = 0; k < 3; ++k)
    if (outs[k])
      FNO_HIP(hipMemcpyAsync(outs[k], res_ + tblocks_[k].offset, tblocks_[k].size * sizeof(double),
                             dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, eng->stream));
  double E = energy();
  if (ec) *ec = E;
  FNO_HIP(hipStreamSynchronize(eng->stream));
}

// MP-style starting amplitudes: two Jacobi steps from zero.  The first gives
// MP2 doubles; the second gives T3 = R3(T2 = MP2) / D3 (the MP2 drivers of the
// triples equations) and the next correction of T2.
void Context::plain_guess() {
  Engine& e = *eng;
  launch_fill(amp_, 0.0, nt_, e.stream);
  for (int s = 0; s < 2; ++s) {
    residual();
    launch_jacobi(amp_, res_, den_, nullptr, nt_, e.stream);
  }
}

double Context::t3_rms(const double* x) {
  const int64_t n3 = tblocks_[2].size;
  const double s = n3 ? std::sqrt(dot(x, x, n3) / (double)n3) : 0.0;
  return s > 0 ? s : 1.0;
}

namespace {
// device copy of the working-space orbital energies (occupied then virtual)
double* upload_eps(const std::vector<double>& fock, int n) {
  std::vector<double> eps(n);
  for (int p = 0; p < n; ++p) eps[p] = fock[(size_t)p * n + p];
  double* d = nullptr;
  FNO_HIP(hipMalloc(&d, n * sizeof(double)));
  FNO_HIP(hipMemcpy(d, eps.data(), n * sizeof(double), hipMemcpyHostToDevice));
  return d;
}
}  // namespace

// t3 = x + sx y0 and the shifted T3 denominators from the network (BF16
// inference), in chunks of 2^20 elements
void Context::learned_t3(const double* x, double sx, double* t3, double* den3) {
  Engine& e = *eng;
  Mlp& m = *guess_model;
  FNO_REQUIRE(m.device == device, kEINVAL, "the guess model lives on another device");
  const int64_t n3 = tblocks_[2].size, chunk = 1 << 20;
  const int64_t cn = std::max<int64_t>(std::min(n3, chunk), 1);
  float *feat = nullptr, *Y = nullptr;
  double* deps = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(e.stream);
    if (feat) (void)hipFree(feat);
    if (Y) (void)hipFree(Y);
    if (deps) (void)hipFree(deps);
  };
  try {
    FNO_HIP(hipMalloc(&feat, (size_t)cn * Mlp::F * sizeof(float)));
    FNO_HIP(hipMalloc(&Y, (size_t)cn * Mlp::O * sizeof(float)));
    deps = upload_eps(fock, nocc + nvir);
    for (int64_t r0 = 0; r0 < n3; r0 += chunk) {
      const int64_t c = std::min(chunk, n3 - r0);
      mlp::features(e.tables, nocc, nvir, x, den3, deps, sx, nullptr, r0, c, feat, nullptr, nullptr, nullptr,
                    e.stream);
      m.predict_bf16(feat, c, Y, e.stream);
      mlp::apply_guess(t3 + r0, x + r0, den3 + r0, Y, sx, c, e.stream);
    }
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

void Context::ml_collect(Mlp& m, int64_t max_samples) {
  FNO_REQUIRE(cc_done, kESTATE, "training samples need a converged fno_ccsdt");
  FNO_REQUIRE(m.device == device, kEINVAL, "the network lives on another device");
  FNO_REQUIRE(max_samples > 0, kEINVAL, "max_samples must be positive");
  Engine& e = *eng;
  const Block& b3 = tblocks_[2];
  const int64_t n3 = b3.size;
  const int n = nocc + nvir;
  std::vector<double*> tmp;
  auto dalloc = [&](int64_t k) {
    double* p = nullptr;
    FNO_HIP(hipMalloc(&p, (size_t)std::max<int64_t>(k, 1) * sizeof(double)));
    tmp.push_back(p);
    return p;
  };
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(e.stream);
    for (double* p : tmp) (void)hipFree(p);
  };
  try {
    double* conv = dalloc(nt_);
    FNO_HIP(hipMemcpyAsync(conv, amp_, nt_ * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    // dressed one-body diagonal at the converged amplitudes (F3_oo, F3_vv)
    residual();
    std::vector<double> foo((size_t)nocc * nocc), fvv((size_t)nvir * nvir), fd(n);
    FNO_HIP(hipMemcpyAsync(foo.data(), e.get("F3_oo")->d, foo.size() * sizeof(double), hipMemcpyDeviceToHost,
                           e.stream));
    FNO_HIP(hipMemcpyAsync(fvv.data(), e.get("F3_vv")->d, fvv.size() * sizeof(double), hipMemcpyDeviceToHost,
                           e.stream));
    FNO_HIP(hipStreamSynchronize(e.stream));
    for (int i = 0; i < nocc; ++i) fd[i] = foo[(size_t)i * nocc + i];
    for (int a = 0; a < nvir; ++a) fd[nocc + a] = fvv[(size_t)a * nvir + a];
    double* dfd = dalloc(n);
    FNO_HIP(hipMemcpy(dfd, fd.data(), n * sizeof(double), hipMemcpyHostToDevice));
    double* deps = upload_eps(fock, n);
    tmp.push_back(deps);
    // the MP-style guess x
    plain_guess();
    double* x = dalloc(n3);
    FNO_HIP(hipMemcpyAsync(x, amp_ + b3.offset, n3 * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    FNO_HIP(hipMemcpyAsync(amp_, conv, nt_ * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    const double sx = t3_rms(x);
    // evenly strided sample of the elements
    const int64_t ns = std::min(max_samples, n3);
    int64_t* idx = nullptr;
    if (ns < n3) {
      std::vector<int64_t> h(ns);
      for (int64_t r = 0; r < ns; ++r) h[r] = (int64_t)((double)r * (double)n3 / (double)ns);
      idx = (int64_t*)dalloc(ns);
      FNO_HIP(hipMemcpy(idx, h.data(), ns * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    float *X = nullptr, *T = nullptr;
    m.reserve(ns, &X, &T);
    mlp::features(e.tables, nocc, nvir, x, den_ + b3.offset, deps, sx, idx, 0, ns, X, conv + b3.offset, dfd, T,
                  e.stream);
    FNO_HIP(hipStreamSynchronize(e.stream));
    m.commit(ns);
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

int Context::ccsdt(const CCOptions& opt, double* ec, double* et, int* iters, double* rn) {
  FNO_REQUIRE(loaded, kESTATE, "no Hamiltonian loaded");
  FNO_REQUIRE(opt.max_iter > 0 && opt.diis_n >= 0 && opt.diis_n <= 16, kEINVAL, "bad solver options");
  if (!cc_ready) setup_cc();
  Engine& e = *eng;
  launch_fill(amp_, 0.0, nt_, e.stream);
  const int m = opt.diis_n;
  std::vector<double*> ht(std::max(m, 1)), he(std::max(m, 1));
  // history vectors at an even stride, so that each starts 16-byte aligned
  const int64_t ldh = (nt_ + 1) / 2 * 2;
  double* hist = alloc(2 * (int64_t)std::max(m, 1) * ldh);
  for (int i = 0; i < std::max(m, 1); ++i) {
    ht[i] = hist + (int64_t)i * ldh;
    he[i] = hist + (int64_t)(std::max(m, 1) + i) * ldh;
  }
  double* dcoef = alloc(32);
  double* dB = alloc(16 * 16);  // error overlaps indexed by slot
  std::vector<int> order;       // history slots, oldest first
  double e_old = energy();
  double rnorm = INFINITY, de = 0;
  trace_e.clear();
  trace_r.clear();
  int it = 0, status = kENOCONV;
  e.prec = opt.prec;
  double* dres = alloc(2 + 16);  // |r|^2, then the overlaps of the new error vector
  const int mm = std::max(m, 1);
  FNO_REQUIRE(diis_step_partials(mm) <= 256 * 1024, kEINVAL, "DIIS partial sums exceed the scratch buffer");
  // learned guess: after two plain Jacobi iterations the amplitudes are the
  // MP-style guess.  At the third iteration the residual is evaluated at the
  // plain guess and at the learned one (the network corrects the T3 block and
  // shifts the T3 Jacobi denominators); the smaller residual norm wins and the
  // iteration continues from it.  The extra evaluation counts as an iteration.
  FNO_REQUIRE(opt.guess == 0 || (opt.guess == 1 && guess_model != nullptr), kEINVAL,
              "guess = 1 needs a guess model (fno_set_guess_model)");
  const Block& b3 = tblocks_[2];
  double* xg = nullptr;    // plain T3 guess
  double* dkeep = nullptr;  // plain T3 denominators
  last_guess_accepted = false;
  auto restore_den = [&]() {
    if (dkeep) FNO_HIP(hipMemcpyAsync(den_ + b3.offset, dkeep, b3.size * sizeof(double), hipMemcpyDeviceToDevice,
                                      e.stream));
  };
  auto release_guess = [&]() {
    FNO_HIP(hipStreamSynchronize(e.stream));
    for (double* q : {xg, dkeep})
      if (q) {
        owned_.erase(std::remove(owned_.begin(), owned_.end(), q), owned_.end());
        FNO_HIP(hipFree(q));
      }
    xg = dkeep = nullptr;
  };
  // the next iteration's residual is enqueued before the host waits for this
  // iteration's energy, so the graph submission overlaps the tail of the work
  // instead of leaving the device idle (when the loop stops there, that
  // residual is left unused: amplitudes and reported norms are unaffected)
  bool ahead = false;
  for (it = 1; it <= opt.max_iter; ++it) {
    if (ahead) {
      ahead = false;
    } else if (opt.guess == 1 && it == 3 && b3.size > 0 && it + 1 <= opt.max_iter) {
      // residual at the plain guess, kept aside
      residual();
      double* rplain = alloc(nt_);
      FNO_HIP(hipMemcpyAsync(rplain, res_, nt_ * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
      const double rn_plain = std::sqrt(dot(res_, res_, nt_));
      // residual at the learned guess
      xg = alloc(b3.size);
      dkeep = alloc(b3.size);
      FNO_HIP(hipMemcpyAsync(xg, amp_ + b3.offset, b3.size * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
      FNO_HIP(hipMemcpyAsync(dkeep, den_ + b3.offset, b3.size * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
      learned_t3(xg, t3_rms(xg), amp_ + b3.offset, den_ + b3.offset);
      residual();
      const double rn_learned = std::sqrt(dot(res_, res_, nt_));
      if (rn_learned < rn_plain) {
        last_guess_accepted = true;
      } else {
        // the plain guess wins: its amplitudes, denominators and residual
        FNO_HIP(hipMemcpyAsync(amp_ + b3.offset, xg, b3.size * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
        restore_den();
        FNO_HIP(hipMemcpyAsync(res_, rplain, nt_ * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
      }
      FNO_HIP(hipStreamSynchronize(e.stream));
      owned_.erase(std::remove(owned_.begin(), owned_.end(), rplain), owned_.end());
      FNO_HIP(hipFree(rplain));
      order.clear();  // the DIIS history restarts from the chosen guess
      ++it;           // the extra residual evaluation of the guess comparison
    } else {
      residual();
    }
    int slot;
    if ((int)order.size() < mm) {
      slot = (int)order.size();
    } else {
      slot = order.front();
      order.erase(order.begin());
    }
    order.push_back(slot);
    // the Jacobi step into the history slot, its error vector, |r|^2 and every
    // overlap <e_s|e_slot> in one pass; the DIIS system is solved on the
    // device, so the host does not wait here: it reads |r|^2 with the energy,
    // after the next residual has been enqueued
    launch_diis_step(amp_, res_, den_, ht[slot], he[0], ldh, slot, m > 0 ? mm : 0, nt_, scratch_, dres, dres + 2,
                     e.stream);
    FNO_HIP(hipMemcpyAsync(pinned() + 1, dres, sizeof(double), hipMemcpyDeviceToHost, e.stream));
    const bool extrap = m > 0 && it >= opt.diis_start && order.size() >= 2;
    if (m > 0) {
      DiisSlots ds;
      ds.k = (int)order.size();
      for (int a = 0; a < ds.k; ++a) ds.slot[a] = order[a];
      launch_diis(dB, dres + 2, slot, ds, extrap, mm, dcoef, e.stream);
    }
    if (extrap)
      launch_combine(amp_, ht[0], ldh, dcoef, mm, 1.0, 0.0, nt_, e.stream);
    else
      launch_axpby(amp_, ht[slot], 1.0, 0.0, nt_, e.stream);
    energy_async();
    if (it < opt.max_iter && !(opt.guess == 1 && it + 1 == 3)) {
      residual(true);
      ahead = true;
    }
    FNO_HIP(hipEventSynchronize(e_ready_));
    rnorm = std::sqrt(host_pin_[1]);
    if (!std::isfinite(rnorm)) {
      FNO_HIP(hipStreamSynchronize(e.stream));
      e.prec = Prec::FP64;
      restore_den();
      release_guess();
      throw Error(kENONFINITE, "non-finite residual at iteration " + std::to_string(it));
    }
    const double E = host_pin_[0];
    de = E - e_old;
    e_old = E;
    trace_e.push_back(E);
    trace_r.push_back(rnorm);
    if (rnorm < opt.r_tol && std::fabs(de) < opt.e_tol) {
      status = kOK;
      break;
    }
    // FP32 / split-BF16 triples products leave a residual floor (rounding of
    // the products, far above FP64's): the solve has converged when the
    // energy is stationary and the norm has stopped falling within a factor
    // 100 of r_tol (its last four values within 25% of each other)
    if (opt.prec != Prec::FP64 && trace_r.size() >= 4 && std::fabs(de) < opt.e_tol && rnorm < 100.0 * opt.r_tol) {
      const auto b = trace_r.end() - 4;
      const double hi = *std::max_element(b, trace_r.end()), lo = *std::min_element(b, trace_r.end());
      if (hi <= 1.25 * lo) {
        status = kOK;
        break;
      }
    }
  }
  e.prec = Prec::FP64;
  restore_den();
  release_guess();
  // release the DIIS history
  FNO_HIP(hipStreamSynchronize(e.stream));
  e.flush_timers(cc_prog_);
  owned_.erase(std::remove(owned_.begin(), owned_.end(), hist), owned_.end());
  owned_.erase(std::remove(owned_.begin(), owned_.end(), dcoef), owned_.end());
  owned_.erase(std::remove(owned_.begin(), owned_.end(), dB), owned_.end());
  owned_.erase(std::remove(owned_.begin(), owned_.end(), dres), owned_.end());
  FNO_HIP(hipFree(hist));
  FNO_HIP(hipFree(dcoef));
  FNO_HIP(hipFree(dB));
  FNO_HIP(hipFree(dres));
  e_corr = e_old;
  cc_done = true;
  if (ec) *ec = e_old;
  if (et) *et = e_ref + e_old;
  if (iters) *iters = std::min(it, opt.max_iter);
  if (rn) *rn = rnorm;
  return status;
}

}  // namespace fno

// EOM-CCSDT sigma vectors (IP, EA, DIP, DEA) and the block Davidson solver.
//
// sigma = <mu| [H-bar, R] |0> over the R space of the variant (eqs 1-4); the
// term tables come from the ground-state residual by differentiation along
// R placed in continuum-orbital blocks (see codegen/eom_jvp.py).  The
// ground-state intermediates (dressed integrals, F3_*, W3_*, ...) are built
// once at the converged amplitudes and reused by every sigma evaluation.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>

#include "eom_space.hpp"
#include "linalg.hpp"

namespace fno {

#include "eom_dea_terms.inc"
#include "eom_dip_terms.inc"
#include "eom_ea_terms.inc"
#include "eom_ip_terms.inc"

namespace {
template <typename T, size_t N>
constexpr int count(const T (&)[N]) {
  return (int)N;
}

std::pair<std::string, std::string> split_decl2(const char* d) {
  std::string s(d);
  size_t c = s.find(':');
  auto trim = [](std::string x) {
    size_t a = x.find_first_not_of(' '), b = x.find_last_not_of(' ');
    return a == std::string::npos ? std::string() : x.substr(a, b - a + 1);
  };
  return {trim(s.substr(0, c)), trim(s.substr(c + 1))};
}

#define FNO_EOM_TABLES(V)                                                                                   \
  EomTables{kEom##V##Decl,     count(kEom##V##Decl),  kEom##V##Views,  count(kEom##V##Views),            \
            kEom##V##Blocks,   kEom##V##Sign,         kEom##V##In,     kEom##V##Out,                     \
            count(kEom##V##In), kEom##V##Zero,        count(kEom##V##Zero), kEom##V##Terms,              \
            count(kEom##V##Terms), kEom##V##PrimDecl, count(kEom##V##PrimDecl), kEom##V##Prep,           \
            count(kEom##V##Prep)}

// the left-hand program: adjoint tensors, inputs (adjoints of the sigma
// blocks), outputs (adjoints of the R blocks), zero list and terms; views
// and T-only intermediates are those of the right-hand program
#define FNO_EOM_LTABLES(V)                                                                                  \
  EomTables{kEom##V##LDecl,     count(kEom##V##LDecl), kEom##V##Views,  count(kEom##V##Views),           \
            kEom##V##Blocks,    kEom##V##Sign,         kEom##V##LIn,    kEom##V##LOut,                    \
            count(kEom##V##LIn), kEom##V##LZero,       count(kEom##V##LZero), kEom##V##LTerms,           \
            count(kEom##V##LTerms), kEom##V##PrimDecl, count(kEom##V##PrimDecl), kEom##V##Prep,          \
            count(kEom##V##Prep)}

EomTables tables_for(int kind, bool left = false) {
  switch (kind) {
    case 1: return left ? FNO_EOM_LTABLES(IP) : FNO_EOM_TABLES(IP);
    case 2: return left ? FNO_EOM_LTABLES(DIP) : FNO_EOM_TABLES(DIP);
    case 3: return left ? FNO_EOM_LTABLES(EA) : FNO_EOM_TABLES(EA);
    case 4: return left ? FNO_EOM_LTABLES(DEA) : FNO_EOM_TABLES(DEA);
    default: throw Error(kEINVAL, "unknown EOM variant");
  }
}

}  // namespace

void Context::release_eom() {
  if (!eom_) return;
  Engine& e = *eng;
  FNO_HIP(hipStreamSynchronize(e.stream));
  for (auto& name : eom_->created) e.drop(name);
  if (eom_->diag) {
    owned_.erase(std::remove(owned_.begin(), owned_.end(), eom_->diag), owned_.end());
    FNO_HIP(hipFree(eom_->diag));
  }
  eom_.reset();
}

void Context::setup_eom(int kind, int nb) {
  FNO_REQUIRE(cc_ready, kESTATE, "EOM needs ground-state amplitudes");
  FNO_REQUIRE(nb >= 1, kEINVAL, "bad EOM block size");
  if (eom_ && eom_->kind == kind && eom_->nb == nb && eom_->ready) return;
  release_eom();
  Engine& e = *eng;
  sz_.n['b'] = nb;
  auto sp = std::make_unique<EomSpace>();
  sp->kind = kind;
  sp->nb = nb;
  sp->tab = tables_for(kind);
  sp->ltab = tables_for(kind, true);
  const EomTables& t = sp->tab;
  auto make = [&](const char* decl) {
    if (!decl[0]) return;
    auto d = split_decl2(decl);
    FNO_REQUIRE(!e.has(d.first), kEDEVICE, "EOM tensor already exists: " + d.first);
    e.create(d.first, d.second, sz_);
    sp->created.push_back(d.first);
  };
  for (int i = 0; i < t.ndecl; ++i) make(t.decl[i]);
  for (int i = 0; i < t.nprim_decl; ++i) make(t.prim_decl[i]);
  for (int i = 0; i < t.nviews; ++i) {
    std::string s(t.views[i]);
    if (s.empty()) continue;
    size_t eq = s.find('='), lp = s.find('('), rp = s.find(')');
    std::string name = s.substr(0, eq), par = s.substr(eq + 1, lp - eq - 1);
    name.erase(std::remove(name.begin(), name.end(), ' '), name.end());
    par.erase(std::remove(par.begin(), par.end(), ' '), par.end());
    std::vector<std::pair<int, int>> rng;
    for (char c : s.substr(lp + 1, rp - lp - 1)) {
      if (c == 'o') rng.push_back({0, nocc});
      if (c == 'v') rng.push_back({nocc, nvir});
      if (c == 'n') rng.push_back({0, nocc + nvir});
    }
    FNO_REQUIRE(!e.has(name), kEDEVICE, "EOM view already exists: " + name);
    e.view(name, e.get(par), rng);
    sp->created.push_back(name);
  }
  // R-vector layout: packed blocks in rank order
  sp->dim = 0;
  for (int b = 0; b < t.nblocks; ++b) {
    Block B;
    B.nh = t.blocks[b][0];
    B.np = t.blocks[b][1];
    B.name = t.in[b];
    B.size = (int64_t)binom_host(nocc, B.nh) * (int64_t)binom_host(nvir, B.np);
    FNO_REQUIRE(B.size * nb == e.get(t.in[b])->elems && B.size * nb == e.get(t.out[b])->elems, kEDEVICE,
                "EOM block layout mismatch");
    B.offset = sp->dim;
    sp->dim += B.size;
    sp->blocks.push_back(B);
  }
  // ground-state intermediates at the current amplitudes, then the T-only
  // intermediates of the quadruples projection (DIP, DEA)
  residual();
  e.prec = Prec::FP64;
  {
    CacheScope cache(e, {"T2", "T3"});
    for (int i = 0; i < t.nprep; ++i)
      if (t.prep[i][0]) e.term(t.prep[i]);
  }
  // diagonal for the preconditioner and the guesses: the one-body part of
  // H-bar at the CC amplitudes (the dressed Fock blocks F3_oo, F3_vv of the
  // triples equations), summed over a block's particles minus its holes
  sp->diag = alloc(sp->dim);
  const int n = nocc + nvir;
  std::vector<double> eo(nocc), ev(nvir);
  {
    std::vector<double> foo((size_t)nocc * nocc), fvv((size_t)nvir * nvir);
    FNO_HIP(hipMemcpy(foo.data(), e.get("F3_oo")->d, foo.size() * sizeof(double), hipMemcpyDeviceToHost));
    FNO_HIP(hipMemcpy(fvv.data(), e.get("F3_vv")->d, fvv.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int i = 0; i < nocc; ++i) eo[i] = foo[(size_t)i * nocc + i];
    for (int a = 0; a < nvir; ++a) ev[a] = fvv[(size_t)a * nvir + a];
  }
  double* d_e = alloc(n);
  FNO_HIP(hipMemcpy(d_e, eo.data(), nocc * sizeof(double), hipMemcpyHostToDevice));
  FNO_HIP(hipMemcpy(d_e + nocc, ev.data(), nvir * sizeof(double), hipMemcpyHostToDevice));
  for (auto& B : sp->blocks) {
    MatDim md{};
    int q = 0;
    if (B.nh > 0) {
      md.grp[q].g = B.nh;
      md.grp[q].n = nocc;
      md.grp[q].count = (int64_t)binom_host(nocc, B.nh);
      for (int s = 0; s < B.nh; ++s) md.grp[q].letter[s] = (int8_t)s;
      ++q;
    }
    if (B.np > 0) {
      md.grp[q].g = B.np;
      md.grp[q].n = nvir;
      md.grp[q].count = (int64_t)binom_host(nvir, B.np);
      for (int s = 0; s < B.np; ++s) md.grp[q].letter[s] = (int8_t)(B.nh + s);
      ++q;
    }
    md.ngroups = q;
    md.size = B.size;
    launch_denominators(e.tables, md, B.nh, d_e, d_e + nocc, sp->diag + B.offset, e.stream);
    launch_axpby(sp->diag + B.offset, sp->diag + B.offset, -1.0, 0.0, B.size, e.stream);
  }
  owned_.erase(std::remove(owned_.begin(), owned_.end(), d_e), owned_.end());
  FNO_HIP(hipStreamSynchronize(e.stream));
  FNO_HIP(hipFree(d_e));
  sp->ready = true;
  eom_ = std::move(sp);
}

size_t Context::eom_size(int kind) {
  FNO_REQUIRE(loaded, kESTATE, "no Hamiltonian loaded");
  const EomTables t = tables_for(kind);
  int64_t d = 0;
  for (int b = 0; b < t.nblocks; ++b)
    d += (int64_t)binom_host(nocc, t.blocks[b][0]) * (int64_t)binom_host(nvir, t.blocks[b][1]);
  return (size_t)d;
}

// The adjoint tensors of the left-hand program, created on first use.
static void ensure_left(Engine& e, Context::EomSpace& sp, const SpaceSizes& sz) {
  if (sp.left_made) return;
  const EomTables& t = sp.ltab;
  for (int i = 0; i < t.ndecl; ++i) {
    auto d = split_decl2(t.decl[i]);
    FNO_REQUIRE(!e.has(d.first), kEDEVICE, "EOM tensor already exists: " + d.first);
    e.create(d.first, d.second, sz);
    sp.created.push_back(d.first);
  }
  for (int b = 0; b < t.nblocks; ++b)
    FNO_REQUIRE(sp.blocks[b].size * sp.nb == e.get(t.in[b])->elems &&
                    sp.blocks[b].size * sp.nb == e.get(t.out[b])->elems,
                kEDEVICE, "EOM left block layout mismatch");
  sp.left_made = true;
}

// sigma_j = (H-bar - E_CC) r_j (left: sigma_j^T = r_j^T (H-bar - E_CC), the
// transposed program) for `count` <= nb device vectors (packed R layout,
// leading dimensions ldr / lds); the block tensors hold nb vectors each,
// those beyond `count` are zero.
static void eom_apply(Context& c, Engine& e, Context::EomSpace& sp, const double* r, int64_t ldr, int count,
                      double* sigma, int64_t lds, Prec prec, bool left = false) {
  const EomTables& t = left ? sp.ltab : sp.tab;
  SigmaGraph& g = left ? sp.lg : sp.rg;
  FNO_REQUIRE(!left || sp.left_made, kESTATE, "left-hand EOM tensors not set up");
  FNO_REQUIRE(count >= 1 && count <= sp.nb, kEINVAL, "bad EOM block count");
  for (int b = 0; b < t.nblocks; ++b) {
    const int64_t sz = sp.blocks[b].size;
    double* in = e.get(t.in[b])->d;
    launch_scale_rows(in, sz, r + sp.blocks[b].offset, ldr, (double)t.sign[b], sz, count, sp.nb, e.stream);
  }
  auto sweep = [&]() {
    std::vector<Tensor*> cleared;
    for (int i = 0; i < t.nzero; ++i) cleared.push_back(e.get(t.zero[i]));
    e.zero_many(cleared);
    e.stats.clear();
    e.record = true;
    // the R blocks are fixed during one sigma: share their expansions
    std::vector<std::string> inputs;
    for (int b = 0; b < t.nblocks; ++b) inputs.push_back(t.in[b]);
    CacheScope cache(e, inputs);
    for (int i = 0; i < t.nterms; ++i) {
      std::string s(t.terms[i]);
      // contractions that read or write the R3 block run in the requested precision
      bool tri = false;
      for (int b = 0; b < t.nblocks; ++b)
        if (sp.blocks[b].nh + sp.blocks[b].np >= 5) {
          tri |= s.find(std::string(t.in[b]) + "[") != std::string::npos;
          tri |= s.rfind(std::string(t.out[b]) + "[", 0) == 0;
        }
      e.prec = tri ? prec : Prec::FP64;
      e.term(s);
    }
    e.prec = Prec::FP64;
    e.record = false;
    double tf = 0, af = 0;
    for (auto& st : e.stats) {
      af += st.flops;
      for (int b = 0; b < t.nblocks; ++b)
        if (sp.blocks[b].nh + sp.blocks[b].np >= 5 &&
            (st.term.find(std::string(t.in[b]) + "[") != std::string::npos ||
             st.term.rfind(std::string(t.out[b]) + "[", 0) == 0)) {
          tf += st.flops;
          break;
        }
    }
    sp.sweep_tri = tf;
    sp.sweep_all = af;
  };
  const bool graphs = c.use_graphs;
  if (graphs && g.prog.valid() && g.prog.epoch == e.epoch && g.prog.prec == (int)prec &&
      g.prog.profiled == e.profile && g.prog.filter == e.profile_filter) {
    e.replay(g.prog);
  } else {
    g.prog.clear();
    bool done = false;
    if (graphs && g.stable && g.stable_epoch == e.epoch && g.stable_prec == (int)prec &&
        g.stable_profiled == e.profile && g.stable_filter == e.profile_filter) {
      e.begin_record(g.prog);
      g.prog.prec = (int)prec;
      bool recorded = false;
      try {
        sweep();
        e.end_record(g.prog);
        recorded = true;
      } catch (const Error&) {
        e.abort_record();
        e.prec = Prec::FP64;
        g.stable = false;
      }
      if (recorded && g.prog.valid()) {
        e.replay(g.prog);
        done = true;
      }
    }
    if (!done) {
      const uint64_t before = e.epoch;
      sweep();
      g.stable = e.epoch == before;
      g.stable_epoch = e.epoch;
      g.stable_prec = (int)prec;
      g.stable_profiled = e.profile;
      g.stable_filter = e.profile_filter;
    }
  }
  for (int b = 0; b < t.nblocks; ++b) {
    const int64_t sz = sp.blocks[b].size;
    const double* out = e.get(t.out[b])->d;
    launch_scale_rows(sigma + sp.blocks[b].offset, lds, out, sz, (double)t.sign[b], sz, count, count, e.stream);
  }
  c.last_triples_flops += sp.sweep_tri;  // summed over the sweeps of a solve (reset by the caller)
  c.last_all_flops += sp.sweep_all;
}

void Context::eom_sigma(int kind, Prec p, const double* r, double* sigma, size_t len, bool dev, bool left) {
  FNO_REQUIRE(cc_ready, kESTATE, "EOM sigma needs amplitudes (fno_ccsdt or fno_set_amplitudes)");
  FNO_REQUIRE(len == eom_size(kind), kEINVAL, "R vector length mismatch");
  if (eom_) eom_->ready = eom_->ready && eom_->kind == kind;
  // amplitudes may have been changed through fno_set_amplitudes: rebuild the intermediates
  release_eom();
  setup_eom(kind, 1);
  Engine& e = *eng;
  if (left) ensure_left(e, *eom_, sz_);
  last_triples_flops = last_all_flops = 0;
  if (dev) {
    eom_apply(*this, e, *eom_, r, (int64_t)len, 1, sigma, (int64_t)len, p, left);
    FNO_HIP(hipStreamSynchronize(e.stream));
    return;
  }
  double* dr = alloc((int64_t)len);
  double* ds = alloc((int64_t)len);
  FNO_HIP(hipMemcpyAsync(dr, r, len * sizeof(double), hipMemcpyHostToDevice, e.stream));
  eom_apply(*this, e, *eom_, dr, (int64_t)len, 1, ds, (int64_t)len, p, left);
  FNO_HIP(hipMemcpyAsync(sigma, ds, len * sizeof(double), hipMemcpyDeviceToHost, e.stream));
  FNO_HIP(hipStreamSynchronize(e.stream));
  FNO_HIP(hipFree(dr));
  FNO_HIP(hipFree(ds));
  owned_.erase(std::remove(owned_.begin(), owned_.end(), dr), owned_.end());
  owned_.erase(std::remove(owned_.begin(), owned_.end(), ds), owned_.end());
}

// Block Davidson for the lowest right eigenpairs (by real part) of the
// nonsymmetric EOM matrix.  Subspace vectors and sigma vectors live on the
// device; the small projected matrix G = V^T S is diagonalised on the host.
// The solver is resumable: dav_sigma issues the sigma vectors of the pending
// subspace vectors on the context's stream without waiting, dav_update does
// one iteration's host work, so that several contexts can be driven in
// lockstep with their device work overlapping (fno_batch_eom).

Context::Davidson* Context::dav_begin(int kind, const EOMOptions& opt) {
  FNO_REQUIRE(cc_done, kESTATE, "fno_eom needs a converged fno_ccsdt first");
  FNO_REQUIRE(opt.nroots >= 1 && opt.max_iter >= 1, kEINVAL, "bad EOM options");
  release_eom();
  // sigma vectors are computed in blocks of up to nroots (at most 16) vectors
  setup_eom(kind, std::min(std::max(opt.block > 0 ? opt.block : opt.nroots, 1), 16));
  EomSpace& sp = *eom_;
  Engine& e = *eng;
  if (opt.left) ensure_left(e, sp, sz_);
  auto d = std::make_unique<Davidson>();
  d->kind = kind;
  d->opt = opt;
  d->dim = sp.dim;
  d->nroots = opt.nroots;
  FNO_REQUIRE(d->nroots <= d->dim, kEINVAL, "more roots than the EOM space has states");
  FNO_REQUIRE(d->nroots <= 256, kEINVAL, "at most 256 roots");
  d->max_sub = std::min(std::max(opt.max_sub > 0 ? opt.max_sub : 8 * d->nroots, 2 * d->nroots), 512);
  const int64_t dim = d->dim;
  {
    // basis and sigma vectors (max_sub each), Ritz vectors and residual
    // block: refuse up front what the device cannot hold
    size_t free_b = 0, total_b = 0;
    FNO_HIP(hipMemGetInfo(&free_b, &total_b));
    const double need = 8.0 * (double)dim * (2.0 * d->max_sub + 3.0 * d->nroots);
    FNO_REQUIRE(need <= (double)free_b, kENOMEM,
                "Davidson storage needs " + std::to_string(need / 1e9) + " GB, the device has " +
                    std::to_string((double)free_b / 1e9) + " GB free (lower max_sub or nroots)");
  }
  d->V = alloc((int64_t)d->max_sub * dim);
  d->S = alloc((int64_t)d->max_sub * dim);
  d->X = alloc((int64_t)d->nroots * dim);
  d->T = alloc((int64_t)2 * d->nroots * dim);
  const int64_t small = (int64_t)2 * d->nroots * d->max_sub + 64;
  d->gres = alloc(small);
  d->cm = alloc(small);
  d->gws_bytes = (size_t)kMaxSplit * (size_t)d->nroots * (size_t)d->max_sub * sizeof(double);
  d->gws = alloc((int64_t)(d->gws_bytes / sizeof(double)));
  // guesses: unit vectors on the lowest zeroth-order diagonal entries of the
  // principal block, continued into the other blocks when it is too small
  std::vector<double> dall(dim);
  FNO_HIP(hipMemcpy(dall.data(), sp.diag, dim * sizeof(double), hipMemcpyDeviceToHost));
  const int64_t n0 = sp.blocks[0].size;
  std::vector<int64_t> order(dim);
  for (int64_t i = 0; i < dim; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    const bool pa = a < n0, pb = b < n0;
    if (pa != pb) return pa;
    return dall[a] < dall[b];
  });
  for (int k = 0; k < d->nroots; ++k) {
    double* v = d->V + (int64_t)k * dim;
    launch_fill(v, 0.0, dim, e.stream);
    double one = 1.0;
    FNO_HIP(hipMemcpyAsync(v + order[k], &one, sizeof(double), hipMemcpyHostToDevice, e.stream));
    FNO_HIP(hipStreamSynchronize(e.stream));
  }
  d->nv = d->nroots;
  last_triples_flops = last_all_flops = 0;  // summed over the sigma sweeps of this solve
  d->G.assign((size_t)d->max_sub * d->max_sub, 0.0);
  d->trace = std::getenv("FNO_TRACE") != nullptr;
  d->theta.assign(d->nroots, 0.0);
  d->theta_imag.assign(d->nroots, 0.0);
  d->theta_old.assign(d->nroots, INFINITY);
  d->rn.assign(d->nroots, INFINITY);
  dav_ = std::move(d);
  return dav_.get();
}

void Context::dav_sigma(Davidson& d) {
  if (d.done) return;
  EomSpace& sp = *eom_;
  Engine& e = *eng;
  while (d.ns < d.nv) {
    const int cnt = std::min(sp.nb, d.nv - d.ns);
    eom_apply(*this, e, sp, d.V + (int64_t)d.ns * d.dim, d.dim, cnt, d.S + (int64_t)d.ns * d.dim, d.dim, d.opt.prec,
              d.opt.left);
    d.ns += cnt;
  }
}

// a term's GEMMs go into one grouped launch when none has this many tiles
constexpr int64_t kGroupBelowTiles = 512;

void Context::GroupedBuffers::reserve(size_t n) {
  if (n <= items) return;
  drop_graph();
  if (stream) FNO_HIP(hipStreamSynchronize(stream));
  if (pin) (void)hipHostFree(pin);
  if (dev) (void)hipFree(dev);
  pin = dev = nullptr;
  items = 0;
  FNO_HIP(hipHostMalloc(&pin, n * gemm_group_item_bytes(), hipHostMallocDefault));
  FNO_HIP(hipMalloc(&dev, n * gemm_group_item_bytes()));
  if (!queue) FNO_HIP(hipMalloc(&queue, 8 * (size_t)gemm_group_max_launches()));
  items = n;
}

void Context::GroupedBuffers::drop_graph() {
  if (exec) {
    if (stream) (void)hipStreamSynchronize(stream);
    (void)hipGraphExecDestroy(exec);
  }
  exec = nullptr;
  key.clear();
}

Context::GroupedBuffers::~GroupedBuffers() {
  if (stream) (void)hipStreamSynchronize(stream);
  drop_graph();
  if (pin) (void)hipHostFree(pin);
  if (dev) (void)hipFree(dev);
  if (queue) (void)hipFree(queue);
  if (ev_s) (void)hipEventDestroy(ev_s);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  if (stream) (void)hipStreamDestroy(stream);
}

// A round: every active instance applies one block of its pending vectors.
// The R blocks go into (and the sigma blocks out of) each instance's tensors
// on its own stream, outside any graph (their addresses change every round);
// the sweep between them (accumulators cleared, then term by term: every
// instance's expansions on its own stream, the grouped GEMMs on the batch
// stream after all of them, every instance's fold on its stream after those)
// is run from the host the first time a round structure is seen, recorded
// into one hipGraph the second time (when no engine allocated anything in
// between) and replayed while the structure stays the same.
void Context::dav_sigma_grouped(const std::vector<Context*>& cs, const std::vector<Davidson*>& ds,
                                GroupedBuffers& gb) {
  const hipStream_t S = gb.stream;
  FNO_REQUIRE(S != nullptr, kEINVAL, "grouped sigma: no batch stream");
  if (!gb.ev_s) FNO_HIP(hipEventCreateWithFlags(&gb.ev_s, hipEventDisableTiming));
  while (gb.ev.size() < cs.size()) {
    hipEvent_t e = nullptr;
    FNO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    gb.ev.push_back(e);
  }
  for (;;) {
    std::vector<int> act;
    for (size_t i = 0; i < cs.size(); ++i)
      if (!ds[i]->done && ds[i]->ns < ds[i]->nv) act.push_back((int)i);
    if (act.empty()) return;
    const size_t na = act.size();
    std::vector<int> cnt(na);
    std::vector<const EomTables*> tab(na);
    for (size_t j = 0; j < na; ++j) {
      Context& c = *cs[act[j]];
      Davidson& d = *ds[act[j]];
      Engine& e = *c.eng;
      EomSpace& sp = *c.eom_;
      FNO_REQUIRE(!d.opt.left || sp.left_made, kESTATE, "left-hand EOM tensors not set up");
      const EomTables& t = d.opt.left ? sp.ltab : sp.tab;
      tab[j] = &t;
      FNO_REQUIRE(t.nterms == tab[0]->nterms, kEINVAL, "grouped sigma: instances of different EOM kinds");
      cnt[j] = std::min(sp.nb, d.nv - d.ns);
      const double* r = d.V + (int64_t)d.ns * d.dim;
      for (int b = 0; b < t.nblocks; ++b) {
        const int64_t sz = sp.blocks[b].size;
        launch_scale_rows(e.get(t.in[b])->d, sz, r + sp.blocks[b].offset, d.dim, (double)t.sign[b], sz, cnt[j],
                          sp.nb, e.stream);
      }
    }
    const int nterms = tab[0]->nterms;
    gb.reserve((size_t)nterms * na);
    // the structure a recording is valid for
    std::vector<int64_t> key;
    bool profiled = false;  // or graphs off on some context: run from the host
    for (size_t j = 0; j < na; ++j) {
      const Engine& e = *cs[act[j]]->eng;
      profiled = profiled || !cs[act[j]]->use_graphs;
      key.push_back(act[j]);
      key.push_back((int64_t)e.epoch);
      key.push_back((int64_t)ds[act[j]]->opt.prec);
      key.push_back(ds[act[j]]->opt.left ? 1 : 0);
      profiled = profiled || e.profile;
    }
    auto join_to_batch = [&]() {  // S after every instance stream
      for (size_t j = 0; j < na; ++j) {
        FNO_HIP(hipEventRecord(gb.ev[j], cs[act[j]]->eng->stream));
        FNO_HIP(hipStreamWaitEvent(S, gb.ev[j], 0));
      }
    };
    auto fork_from_batch = [&]() {  // every instance stream after S
      FNO_HIP(hipEventRecord(gb.ev_s, S));
      for (size_t j = 0; j < na; ++j) FNO_HIP(hipStreamWaitEvent(cs[act[j]]->eng->stream, gb.ev_s, 0));
    };
    auto sweep = [&]() {
      std::vector<std::unique_ptr<CacheScope>> scope(na);
      struct Reset {
        const std::vector<Context*>& cs;
        const std::vector<int>& act;
        ~Reset() {
          for (int i : act) {
            Engine& e = *cs[i]->eng;
            e.sink = nullptr;
            e.prec = Prec::FP64;
            e.record = false;
          }
        }
      } reset{cs, act};
      for (size_t j = 0; j < na; ++j) {
        Engine& e = *cs[act[j]]->eng;
        const EomTables& t = *tab[j];
        std::vector<Tensor*> cleared;
        for (int i = 0; i < t.nzero; ++i) cleared.push_back(e.get(t.zero[i]));
        e.zero_many(cleared);
        e.stats.clear();
        e.record = true;
        std::vector<std::string> inputs;
        for (int b = 0; b < t.nblocks; ++b) inputs.push_back(t.in[b]);
        scope[j].reset(new CacheScope(e, inputs));
      }
      std::vector<Engine::GemmSink> sink(na);
      const size_t isz = gemm_group_item_bytes();
      for (int k = 0; k < nterms; ++k) {
        std::vector<GemmArgs> all;
        for (size_t j = 0; j < na; ++j) {
          Context& c = *cs[act[j]];
          Engine& e = *c.eng;
          EomSpace& sp = *c.eom_;
          const EomTables& t = *tab[j];
          const std::string s(t.terms[k]);
          bool tri = false;  // contractions that read or write the R3 block run in the requested precision
          for (int b = 0; b < t.nblocks; ++b)
            if (sp.blocks[b].nh + sp.blocks[b].np >= 5) {
              tri |= s.find(std::string(t.in[b]) + "[") != std::string::npos;
              tri |= s.rfind(std::string(t.out[b]) + "[", 0) == 0;
            }
          e.prec = tri ? ds[act[j]]->opt.prec : Prec::FP64;
          e.sink = &sink[j];
          e.term(s);
          e.sink = nullptr;
          all.insert(all.end(), sink[j].gemms.begin(), sink[j].gemms.end());
        }
        // grouped only when every GEMM of the term would leave the device
        // under-filled on its own (the grouped launch joins all instances at
        // the term); otherwise each instance runs its GEMM on its own stream
        // (the same kernel, so the same bits)
        bool group = !all.empty();
        for (const GemmArgs& g : all) group = group && gemm_tiles(g) < kGroupBelowTiles;
        if (group) {
          join_to_batch();
          // each term has its own regions of the item tables: the copies of
          // earlier terms may still be pending when this one is written, and
          // a recording keeps every term's items
          launch_gemm_grouped(all, (char*)gb.pin + (size_t)k * na * isz, (char*)gb.dev + (size_t)k * na * isz,
                              gb.queue, S);
          fork_from_batch();
        }
        for (size_t j = 0; j < na; ++j) {
          Engine& e = *cs[act[j]]->eng;
          if (!group)
            for (const GemmArgs& g : sink[j].gemms) launch_gemm(g, e.stream);
          for (auto& f : sink[j].after) f();
          sink[j].gemms.clear();
          sink[j].after.clear();
        }
      }
      for (size_t j = 0; j < na; ++j) scope[j].reset();
    };
    bool ran = false;
    if (!profiled && gb.exec && key == gb.key) {
      join_to_batch();
      FNO_HIP(hipGraphLaunch(gb.exec, S));
      fork_from_batch();
      ++gb.replays;
      ran = true;
    } else if (!profiled && key == gb.seen) {
      // record: the batch stream starts the capture, the instance streams
      // join it through the fork event and leave it through the final join
      gb.drop_graph();
      join_to_batch();  // outside the capture: S after the R blocks are in place
      Program dummy;
      for (int i : act) cs[i]->eng->set_external_record(&dummy);
      hipGraph_t graph = nullptr;
      bool ok = false;
      FNO_HIP(hipStreamBeginCapture(S, hipStreamCaptureModeRelaxed));
      try {
        fork_from_batch();
        sweep();
        join_to_batch();
        ok = true;
      } catch (const Error&) {
        try {  // leave no instance stream inside the (now invalid) capture
          join_to_batch();
        } catch (const Error&) {
        }
      }
      for (int i : act) cs[i]->eng->set_external_record(nullptr);
      const hipError_t st = hipStreamEndCapture(S, &graph);
      if (ok && st == hipSuccess && graph) {
        hipGraphExec_t exec = nullptr;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
          gb.exec = exec;
          gb.key = key;
          ++gb.recordings;
        }
      }
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      if (gb.exec) {
        FNO_HIP(hipGraphLaunch(gb.exec, S));
        fork_from_batch();
        ran = true;
      }
      gb.seen.clear();
    }
    if (!ran) {
      // from the host (the host-written item tables of a recording would be
      // overwritten: drop it)
      gb.drop_graph();
      join_to_batch();
      fork_from_batch();
      sweep();
      std::vector<int64_t> after;
      for (size_t j = 0; j < na; ++j) {
        const Engine& e = *cs[act[j]]->eng;
        after.push_back(act[j]);
        after.push_back((int64_t)e.epoch);
        after.push_back((int64_t)ds[act[j]]->opt.prec);
        after.push_back(ds[act[j]]->opt.left ? 1 : 0);
      }
      gb.seen = after == key ? key : std::vector<int64_t>{};
    }
    for (size_t j = 0; j < na; ++j) {
      Context& c = *cs[act[j]];
      Davidson& d = *ds[act[j]];
      Engine& e = *c.eng;
      EomSpace& sp = *c.eom_;
      const EomTables& t = *tab[j];
      {  // flops of the sweep (a replay has the statistics of the host-run or recorded sweep)
        double tf = 0, af = 0;
        for (auto& st : e.stats) {
          af += st.flops;
          for (int b = 0; b < t.nblocks; ++b)
            if (sp.blocks[b].nh + sp.blocks[b].np >= 5 &&
                (st.term.find(std::string(t.in[b]) + "[") != std::string::npos ||
                 st.term.rfind(std::string(t.out[b]) + "[", 0) == 0)) {
              tf += st.flops;
              break;
            }
        }
        c.last_triples_flops += tf;
        c.last_all_flops += af;
      }
      double* sigma = d.S + (int64_t)d.ns * d.dim;
      for (int b = 0; b < t.nblocks; ++b) {
        const int64_t sz = sp.blocks[b].size;
        launch_scale_rows(sigma + sp.blocks[b].offset, d.dim, e.get(t.out[b])->d, sz, (double)t.sign[b], sz,
                          cnt[j], cnt[j], e.stream);
      }
      d.ns += cnt[j];
    }
  }
}

namespace {
// Block operations of the Davidson solver as FP64 MFMA GEMMs over vectors
// stored one after another (stride dim): each pass streams a block of
// vectors once, whatever the number of roots.
struct DavBlock {
  Engine& e;
  Context::Davidson& d;
  int64_t dim;
  // gres[i][j] = x_i . y_j (i < a, j < b, row-major), a split-K GEMM over dim
  void gram_dev(const double* X, int a, const double* Y, int b) {
    GemmArgs g{};
    g.prec = Prec::FP64;
    g.M = a;
    g.N = b;
    g.K = dim;
    g.A = X;
    g.lda = dim;
    g.a_kfast = true;
    g.B = Y;
    g.ldb = dim;
    g.b_nfast = false;
    g.C = d.gres;
    g.ldc = b;
    g.alpha = 1.0;
    g.beta = 0.0;
    g.tile = -1;
    g.split = gemm_split_factor(g);
    if (g.split > 1) {
      FNO_REQUIRE(gemm_split_bytes(g, g.split) <= d.gws_bytes, kEINVAL, "Davidson split-K workspace too small");
      g.ws = d.gws;
    }
    launch_gemm(g, e.stream);
  }
  void gram(const double* X, int a, const double* Y, int b, std::vector<double>& out) {
    out.assign((size_t)a * b, 0.0);
    if (a == 0 || b == 0) return;
    gram_dev(X, a, Y, b);
    FNO_HIP(hipMemcpyAsync(out.data(), d.gres, out.size() * sizeof(double), hipMemcpyDeviceToHost, e.stream));
    FNO_HIP(hipStreamSynchronize(e.stream));
  }
  // Y_j = alpha * sum_k c[j][k] x_k + beta * Y_j for j < m, k < n (c row-major
  // m x n on the device)
  void combine_dev(double* Y, int m, const double* X, int n, const double* c, double alpha, double beta) {
    if (m == 0) return;
    GemmArgs g{};
    g.prec = Prec::FP64;
    g.M = m;
    g.N = dim;
    g.K = n;
    g.A = c;
    g.lda = n;
    g.a_kfast = true;
    g.B = X;
    g.ldb = dim;
    g.b_nfast = true;
    g.C = Y;
    g.ldc = dim;
    g.alpha = alpha;
    g.beta = beta;
    g.tile = -1;
    g.split = 1;
    launch_gemm(g, e.stream);
  }
  void combine(double* Y, int m, const double* X, int n, const std::vector<double>& c, double alpha, double beta) {
    if (m == 0) return;
    FNO_REQUIRE((int64_t)c.size() == (int64_t)m * n, kEINVAL, "coefficient block size");
    FNO_HIP(hipMemcpyAsync(d.cm, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, e.stream));
    combine_dev(Y, m, X, n, d.cm, alpha, beta);
    FNO_HIP(hipStreamSynchronize(e.stream));
  }
};

// Cholesky-QR of a block of u vectors with Gram matrix M (u x u): rows of
// the returned q x u matrix T give orthonormal vectors T w; a vector whose
// part outside the span of the earlier ones is below tol times its reference
// norm sqrt(ref[p]) is dropped.
std::vector<double> chol_qr(const std::vector<double>& M, int u, const std::vector<double>& ref, double tol,
                            int& q) {
  std::vector<std::vector<double>> rows;
  for (int p = 0; p < u; ++p) {
    std::vector<double> c(rows.size());
    for (size_t s = 0; s < rows.size(); ++s) {
      double t = 0;
      for (int r = 0; r < u; ++r) t += rows[s][r] * M[(size_t)r * u + p];
      c[s] = t;
    }
    double res2 = M[(size_t)p * u + p];
    for (double x : c) res2 -= x * x;
    if (!(res2 > tol * tol * ref[p]) || !(res2 > 1e-300)) continue;
    std::vector<double> t(u, 0.0);
    t[p] = 1.0;
    for (size_t s = 0; s < rows.size(); ++s)
      for (int r = 0; r < u; ++r) t[r] -= c[s] * rows[s][r];
    const double inv = 1.0 / std::sqrt(res2);
    for (double& x : t) x *= inv;
    rows.push_back(std::move(t));
  }
  q = (int)rows.size();
  std::vector<double> out((size_t)q * u);
  for (int s = 0; s < q; ++s)
    for (int r = 0; r < u; ++r) out[(size_t)s * u + r] = rows[s][r];
  return out;
}
}  // namespace

bool Context::dav_update(Davidson& d) {
  if (d.done) return true;
  EomSpace& sp = *eom_;
  Engine& e = *eng;
  const int64_t dim = d.dim;
  const int nroots = d.nroots, max_sub = d.max_sub;
  DavBlock blk{e, d, dim};
  auto vec = [&](double* base, int j) { return base + (int64_t)j * dim; };
  ++d.it;
  int nv = d.nv;
  // G[i][j] = v_i . s_j; only the rows and columns of the vectors added since
  // the last iteration are new
  if (d.gn < nv) {
    const int a = nv - d.gn;
    std::vector<double> rows;
    blk.gram(vec(d.V, d.gn), a, d.S, nv, rows);
    for (int r = 0; r < a; ++r)
      for (int j = 0; j < nv; ++j) d.G[(size_t)(d.gn + r) * max_sub + j] = rows[(size_t)r * nv + j];
    if (d.gn > 0) {
      std::vector<double> cols;
      blk.gram(vec(d.S, d.gn), a, d.V, d.gn, cols);
      for (int r = 0; r < a; ++r)
        for (int i = 0; i < d.gn; ++i) d.G[(size_t)i * max_sub + d.gn + r] = cols[(size_t)r * d.gn + i];
    }
  }
  d.gn = nv;
  std::vector<double> Gs((size_t)nv * nv);
  double gscale = 0;
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      Gs[(size_t)i * nv + j] = d.G[(size_t)i * max_sub + j];
      gscale = std::max(gscale, std::fabs(Gs[(size_t)i * nv + j]));
    }
  std::vector<double> wr, wi;
  FNO_REQUIRE(nonsym_eigvals(nv, Gs, wr, wi), kENOCONV, "subspace eigenproblem failed");
  std::vector<int> idx(nv);
  for (int i = 0; i < nv; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return wr[a] < wr[b]; });
  // Ritz coefficients (unit norm: the basis is orthonormal).  A real
  // eigenvalue takes its eigenvector; the two members of a complex-conjugate
  // pair (adjacent after the sort) take the real and the imaginary part of
  // the pair's eigenvector, which span the same real invariant subspace.
  const double imag_tol = 1e-12 * std::max(gscale, 1.0);
  std::vector<std::vector<double>> Y(nroots);
  std::vector<std::complex<double>> yc;
  int yc_root = -2;
  for (int k = 0; k < nroots; ++k) {
    const int j = idx[k];
    d.theta[k] = wr[j];
    d.theta_imag[k] = wi[j];
    if (std::fabs(wi[j]) <= imag_tol) {
      inverse_iteration(nv, Gs, wr[j], Y[k]);
    } else if (yc_root == k - 1 && wr[idx[k - 1]] == wr[j] && wi[idx[k - 1]] == -wi[j]) {
      Y[k].resize(nv);
      for (int i = 0; i < nv; ++i) Y[k][i] = yc[i].imag();
    } else {
      inverse_iteration_c(nv, Gs, {wr[j], wi[j]}, yc);
      yc_root = k;
      Y[k].resize(nv);
      for (int i = 0; i < nv; ++i) Y[k][i] = yc[i].real();
    }
    double nrm = 0;
    for (double y : Y[k]) nrm += y * y;
    nrm = std::sqrt(nrm);
    if (nrm > 0)
      for (double& y : Y[k]) y /= nrm;
  }
  if (nv + nroots > max_sub) {
    // thick restart: keep the Ritz vectors and those of the previous
    // iteration, orthonormalised in coefficient space; the sigma vectors
    // follow by the same combinations, so nothing is recomputed
    std::vector<std::vector<double>> C;
    const size_t cap = (size_t)std::max(nroots, max_sub - nroots);
    auto keep = [&](std::vector<double> c) {
      if (C.size() >= cap) return;
      c.resize(nv, 0.0);
      for (int pass = 0; pass < 2; ++pass)
        for (const auto& q : C) {
          double t = 0;
          for (int i = 0; i < nv; ++i) t += q[i] * c[i];
          for (int i = 0; i < nv; ++i) c[i] -= t * q[i];
        }
      double nrm = 0;
      for (double x : c) nrm += x * x;
      nrm = std::sqrt(nrm);
      if (nrm > 1e-8) {
        for (double& x : c) x /= nrm;
        C.push_back(std::move(c));
      }
    };
    for (int k = 0; k < nroots; ++k) keep(Y[k]);
    for (const auto& y : d.yold) keep(y);
    const int m = (int)C.size();
    std::vector<double> Cf((size_t)m * nv);
    for (int a = 0; a < m; ++a)
      for (int i = 0; i < nv; ++i) Cf[(size_t)a * nv + i] = C[a][i];
    for (double* base : {d.V, d.S}) {
      blk.combine(d.T, m, base, nv, Cf, 1.0, 0.0);
      FNO_HIP(hipMemcpyAsync(base, d.T, (size_t)m * dim * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    }
    // G' = C G C^T
    std::vector<double> GC((size_t)nv * m, 0.0);
    for (int i = 0; i < nv; ++i)
      for (int b = 0; b < m; ++b) {
        double t = 0;
        for (int j = 0; j < nv; ++j) t += Gs[(size_t)i * nv + j] * C[b][j];
        GC[(size_t)i * m + b] = t;
      }
    for (int a = 0; a < m; ++a)
      for (int b = 0; b < m; ++b) {
        double t = 0;
        for (int i = 0; i < nv; ++i) t += C[a][i] * GC[(size_t)i * m + b];
        d.G[(size_t)a * max_sub + b] = t;
      }
    // Ritz coefficients in the new basis
    for (int k = 0; k < nroots; ++k) {
      std::vector<double> y(m);
      for (int a = 0; a < m; ++a) {
        double t = 0;
        for (int i = 0; i < nv; ++i) t += C[a][i] * Y[k][i];
        y[a] = t;
      }
      Y[k] = std::move(y);
    }
    FNO_HIP(hipStreamSynchronize(e.stream));
    d.nv = d.ns = d.gn = nv = m;
    if (d.trace) std::fprintf(stderr, "[fno] davidson restart: %d vectors kept\n", m);
  }
  // Ritz vectors X = V y and residuals T = S y - theta V y, for all roots in
  // three passes over the basis
  std::vector<double> Yf((size_t)nroots * nv), Yt((size_t)nroots * nv);
  for (int k = 0; k < nroots; ++k)
    for (int i = 0; i < nv; ++i) {
      Yf[(size_t)k * nv + i] = Y[k][i];
      Yt[(size_t)k * nv + i] = -d.theta[k] * Y[k][i];
    }
  blk.combine(d.X, nroots, d.V, nv, Yf, 1.0, 0.0);
  blk.combine(d.T, nroots, d.S, nv, Yf, 1.0, 0.0);
  blk.combine(d.T, nroots, d.V, nv, Yt, 1.0, 1.0);
  std::vector<double> rr;
  blk.gram(d.T, nroots, d.T, nroots, rr);
  bool all_conv = true;
  for (int k = 0; k < nroots; ++k) {
    d.rn[k] = std::sqrt(std::max(rr[(size_t)k * nroots + k], 0.0));
    if (!std::isfinite(d.rn[k])) throw Error(kENONFINITE, "non-finite EOM residual");
    all_conv = all_conv && d.rn[k] < d.opt.r_tol && std::fabs(d.theta[k] - d.theta_old[k]) < d.opt.e_tol;
  }
  if (d.trace) {
    std::fprintf(stderr, "[fno] davidson it %d nv %d", d.it, nv);
    for (int k = 0; k < nroots; ++k)
      std::fprintf(stderr, " | %.10f%s r %.1e", d.theta[k], std::fabs(d.theta_imag[k]) > imag_tol ? "(c)" : "",
                   d.rn[k]);
    std::fprintf(stderr, "\n");
  }
  d.theta_old = d.theta;
  if (all_conv) {
    d.status = kOK;
    d.done = true;
    return true;
  }
  if (d.it >= d.opt.max_iter) {
    d.done = true;
    return true;
  }
  d.yold = Y;
  // new directions: preconditioned residuals of the unconverged roots,
  // orthogonalised against the basis and among themselves (twice: block
  // Gram-Schmidt against V, then Cholesky-QR within the block)
  int u = 0;
  for (int k = 0; k < nroots && nv + u < max_sub; ++k) {
    if (d.rn[k] < d.opt.r_tol) continue;
    launch_precond(vec(d.V, nv + u), vec(d.T, k), sp.diag, d.theta[k], dim, e.stream);
    ++u;
  }
  if (u == 0) return false;
  double* P = vec(d.V, nv);
  std::vector<double> M;
  blk.gram(P, u, P, u, M);
  std::vector<double> ref(u);
  for (int p = 0; p < u; ++p) ref[p] = M[(size_t)p * u + p];
  for (int pass = 0; pass < 2 && u > 0; ++pass) {
    blk.gram_dev(P, u, d.V, nv);
    blk.combine_dev(P, u, d.V, nv, d.gres, -1.0, 1.0);
    blk.gram(P, u, P, u, M);
    int q = 0;
    const std::vector<double> Tq = chol_qr(M, u, ref, pass == 0 ? 1e-8 : 1e-6, q);
    blk.combine(d.T, q, P, u, Tq, 1.0, 0.0);
    FNO_HIP(hipMemcpyAsync(P, d.T, (size_t)q * dim * sizeof(double), hipMemcpyDeviceToDevice, e.stream));
    u = q;
    ref.assign(u, 1.0);
  }
  FNO_HIP(hipStreamSynchronize(e.stream));
  d.nv = nv + u;
  return false;
}

int Context::dav_end(EOMResult& res) {
  if (!dav_) return kESTATE;
  Davidson& d = *dav_;
  res.omega = d.theta;
  res.res_norm = d.rn;
  res.iters = std::min(d.it, d.opt.max_iter);
  res.converged = d.status == kOK;
  if (res.want_vectors) {
    res.vectors.resize((size_t)d.nroots * (size_t)d.dim);
    FNO_HIP(hipMemcpy(res.vectors.data(), d.X, res.vectors.size() * sizeof(double), hipMemcpyDeviceToHost));
  }
  const int st = d.status;
  dav_release();
  return st;
}

void Context::dav_release() {
  if (!dav_) return;
  Davidson& d = *dav_;
  (void)hipStreamSynchronize(eng->stream);
  for (double* p : {d.V, d.S, d.X, d.T, d.gres, d.cm, d.gws}) {
    owned_.erase(std::remove(owned_.begin(), owned_.end(), p), owned_.end());
    (void)hipFree(p);
  }
  dav_.reset();
}

int Context::eom(int kind, const EOMOptions& opt, EOMResult& res) {
  Davidson* d = dav_begin(kind, opt);
  try {
    for (;;) {
      dav_sigma(*d);
      if (dav_update(*d)) break;
    }
  } catch (...) {
    dav_release();
    throw;
  }
  return dav_end(res);
}

}  // namespace fno

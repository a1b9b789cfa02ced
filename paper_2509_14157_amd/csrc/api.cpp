// extern "C" boundary: argument checks, error capture, status codes.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>

#include "../../include/fnocc.h"
#include "context.hpp"
#include "eom_space.hpp"
#include "mlp.hpp"

struct fno_ctx {
  fno::Context* c = nullptr;
  std::string err;
};

namespace {
template <typename F>
int guard(fno_ctx* ctx, F&& f) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  try {
    FNO_HIP(hipSetDevice(ctx->c->device));
    ctx->err.clear();
    return f(*ctx->c);
  } catch (const fno::Error& e) {
    ctx->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return FNO_ENOMEM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return FNO_EDEVICE;
  }
}

fno::Prec to_prec(fno_prec p) {
  switch (p) {
    case FNO_FP64: return fno::Prec::FP64;
    case FNO_FP32: return fno::Prec::FP32;
    case FNO_BF16X3: return fno::Prec::BF16X3;
  }
  throw fno::Error(FNO_EINVAL, "unknown precision");
}
}  // namespace

// ---------------------------------------------------------------- learned guess
struct fno_mlp {
  fno::Mlp* m = nullptr;
  std::string err;
};

namespace {
template <typename F>
int mguard(fno_mlp* h, F&& f) {
  if (!h || !h->m) return FNO_EINVAL;
  try {
    FNO_HIP(hipSetDevice(h->m->device));
    h->err.clear();
    return f(*h->m);
  } catch (const fno::Error& e) {
    h->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return FNO_ENOMEM;
  } catch (const std::exception& e) {
    h->err = e.what();
    return FNO_EDEVICE;
  }
}
}  // namespace


extern "C" {

int fno_create(int hip_device, fno_ctx** out) {
  if (!out) return FNO_EINVAL;
  *out = nullptr;
  auto* ctx = new (std::nothrow) fno_ctx;
  if (!ctx) return FNO_ENOMEM;
  try {
    ctx->c = new fno::Context(hip_device);
  } catch (const fno::Error& e) {
    delete ctx;
    return e.code;
  } catch (...) {
    delete ctx;
    return FNO_EDEVICE;
  }
  *out = ctx;
  return FNO_OK;
}

void fno_destroy(fno_ctx* ctx) {
  if (!ctx) return;
  delete ctx->c;
  delete ctx;
}

const char* fno_last_error(const fno_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int fno_set_stream(fno_ctx* ctx, void* s) {
  return guard(ctx, [&](fno::Context& c) {
    c.set_stream((hipStream_t)s);
    return FNO_OK;
  });
}

int fno_load_hamiltonian(fno_ctx* ctx, int nocc, int nvir, const double* fock, const double* eri, double e_nuc) {
  return guard(ctx, [&](fno::Context& c) {
    c.load(nocc, nvir, fock, eri, e_nuc);
    return FNO_OK;
  });
}

int fno_truncate(fno_ctx* ctx, double occt, int nvir_keep, int* nvir_kept, double* e_mp2, double* occ) {
  return guard(ctx, [&](fno::Context& c) {
    c.truncate(occt, nvir_keep, nvir_kept, e_mp2, occ);
    return FNO_OK;
  });
}

void fno_cc_opts_default(fno_cc_opts* o) {
  if (!o) return;
  o->max_iter = 100;
  o->r_tol = 1e-8;
  o->e_tol = 1e-10;
  o->diis_n = 8;
  o->diis_start = 3;
  o->prec = FNO_FP64;
  o->guess = 0;
}

int fno_ccsdt(fno_ctx* ctx, const fno_cc_opts* opts, double* e_corr, double* e_tot, int* iters, double* res_norm) {
  return guard(ctx, [&](fno::Context& c) {
    fno_cc_opts d;
    fno_cc_opts_default(&d);
    const fno_cc_opts& o = opts ? *opts : d;
    FNO_REQUIRE(o.guess == 0 || o.guess == 1, FNO_EINVAL, "guess must be 0 (zero amplitudes) or 1 (learned)");
    fno::CCOptions co;
    co.max_iter = o.max_iter;
    co.r_tol = o.r_tol;
    co.e_tol = o.e_tol;
    co.diis_n = o.diis_n;
    co.diis_start = o.diis_start;
    co.prec = to_prec(o.prec);
    co.guess = o.guess;
    int st = c.ccsdt(co, e_corr, e_tot, iters, res_norm);
    if (st == FNO_ENOCONV) ctx->err = "CCSDT did not converge within max_iter";
    return st;
  });
}

void fno_eom_opts_default(fno_eom_opts* o) {
  if (!o) return;
  o->nroots = 4;
  o->max_iter = 60;
  o->max_sub = 0;
  o->e_tol = 1e-8;
  o->r_tol = 1e-6;
  o->prec = FNO_FP64;
  o->guess = 0;
  o->precond = 0;
  o->block = 0;
}

namespace {
fno::EOMOptions eom_options(const fno_eom_opts* opts) {
  fno_eom_opts d;
  fno_eom_opts_default(&d);
  const fno_eom_opts& o = opts ? *opts : d;
  FNO_REQUIRE(o.guess == 0 && o.precond == 0, FNO_EINVAL, "unsupported guess/preconditioner option");
  FNO_REQUIRE(o.block >= 0 && o.block <= 16, FNO_EINVAL, "block must be in [0, 16]");
  fno::EOMOptions eo;
  eo.nroots = o.nroots;
  eo.max_iter = o.max_iter;
  eo.max_sub = o.max_sub;
  eo.e_tol = o.e_tol;
  eo.r_tol = o.r_tol;
  eo.prec = to_prec(o.prec);
  eo.block = o.block;
  return eo;
}
}  // namespace

namespace {
int batch_eom(int n, fno_ctx* const* ctxs, fno_eom_kind kind, const fno_eom_opts* opts, double* omega,
              double* res_norm, int* iters, bool grouped) {
  if (n <= 0 || !ctxs || !omega) return FNO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || !ctxs[i]->c) return FNO_EINVAL;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (ctxs[i] == ctxs[j]) {
        ctxs[i]->err = "a context appears twice in the batch";
        return FNO_EINVAL;
      }
  std::vector<fno::Context::Davidson*> d(n, nullptr);
  int failed = -1;
  try {
    FNO_REQUIRE(kind >= FNO_IP && kind <= FNO_DEA, FNO_EINVAL, "unknown EOM kind");
    const fno::EOMOptions eo = eom_options(opts);
    for (int i = 0; i < n; ++i) {
      failed = i;
      ctxs[i]->err.clear();
      FNO_HIP(hipSetDevice(ctxs[i]->c->device));
      FNO_REQUIRE(ctxs[i]->c->cc_done, FNO_ESTATE, "fno_batch_eom needs a converged fno_ccsdt on every context");
      d[i] = ctxs[i]->c->dav_begin((int)kind, eo);
    }
    // lockstep: the sigma work of every instance is issued on its own stream
    // before any host wait (or, grouped, as grouped rounds on one batch
    // stream), then each instance does its subspace step
    std::vector<fno::Context*> cs(n);
    for (int i = 0; i < n; ++i) cs[i] = ctxs[i]->c;
    fno::Context::GroupedBuffers gb;  // owns the batch stream
    if (grouped) {
      for (int i = 1; i < n; ++i)
        FNO_REQUIRE(cs[i]->device == cs[0]->device, FNO_EINVAL, "a grouped batch runs on one device");
      FNO_HIP(hipSetDevice(cs[0]->device));
      FNO_HIP(hipStreamCreate(&gb.stream));
    }
    for (bool all_done = false; !all_done;) {
      if (grouped) {
        failed = 0;
        fno::Context::dav_sigma_grouped(cs, d, gb);
      } else {
        for (int i = 0; i < n; ++i) {
          failed = i;
          if (!d[i]->done) ctxs[i]->c->dav_sigma(*d[i]);
        }
      }
      all_done = true;
      for (int i = 0; i < n; ++i) {
        failed = i;
        if (!d[i]->done) ctxs[i]->c->dav_update(*d[i]);
        all_done = all_done && d[i]->done;
      }
    }
    if (grouped && std::getenv("FNO_TRACE"))
      std::fprintf(stderr, "[fno] grouped sigma rounds: %d recordings, %d replays\n", gb.recordings, gb.replays);
    int status = FNO_OK;
    for (int i = 0; i < n; ++i) {
      failed = i;
      fno::EOMResult r;
      const int st = ctxs[i]->c->dav_end(r);
      for (int k = 0; k < eo.nroots; ++k) {
        omega[(size_t)i * eo.nroots + k] = r.omega[k];
        if (res_norm) res_norm[(size_t)i * eo.nroots + k] = r.res_norm[k];
      }
      if (iters) iters[i] = r.iters;
      if (st != FNO_OK) status = FNO_ENOCONV;
    }
    return status;
  } catch (const fno::Error& e) {
    for (int i = 0; i < n; ++i) ctxs[i]->c->dav_release();
    if (failed >= 0) ctxs[failed]->err = e.what();
    if (failed != 0) ctxs[0]->err = std::string("instance ") + std::to_string(failed) + ": " + e.what();
    return e.code;
  } catch (const std::exception& e) {
    for (int i = 0; i < n; ++i) ctxs[i]->c->dav_release();
    ctxs[0]->err = e.what();
    return FNO_EDEVICE;
  }
}

}  // namespace

int fno_batch_eom(int n, fno_ctx* const* ctxs, fno_eom_kind kind, const fno_eom_opts* opts, double* omega,
                  double* res_norm, int* iters) {
  return batch_eom(n, ctxs, kind, opts, omega, res_norm, iters, false);
}

int fno_batch_eom_grouped(int n, fno_ctx* const* ctxs, fno_eom_kind kind, const fno_eom_opts* opts, double* omega,
                          double* res_norm, int* iters) {
  return batch_eom(n, ctxs, kind, opts, omega, res_norm, iters, true);
}

int fno_eom(fno_ctx* ctx, fno_eom_kind kind, const fno_eom_opts* opts, double* omega, double* e_tot,
            double* res_norm, int* iters) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(kind >= FNO_IP && kind <= FNO_DEA, FNO_EINVAL, "unknown EOM kind");
    FNO_REQUIRE(c.cc_done, FNO_ESTATE, "fno_eom needs a converged fno_ccsdt first");
    FNO_REQUIRE(omega != nullptr, FNO_EINVAL, "omega is required");
    const fno::EOMOptions eo = eom_options(opts);
    fno::EOMResult r;
    int st = c.eom((int)kind, eo, r);
    for (int k = 0; k < eo.nroots; ++k) {
      omega[k] = r.omega[k];
      if (e_tot) e_tot[k] = c.e_ref + c.e_corr + r.omega[k];
      if (res_norm) res_norm[k] = r.res_norm[k];
    }
    if (iters) *iters = r.iters;
    if (st == FNO_ENOCONV) ctx->err = "EOM Davidson did not converge within max_iter";
    return st;
  });
}

int fno_mp2_energies(const fno_ctx* ctx, double* e_full, double* e_trunc) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  if (!ctx->c->truncated) return FNO_ESTATE;
  if (e_full) *e_full = ctx->c->e_mp2_full;
  if (e_trunc) *e_trunc = ctx->c->e_mp2_trunc;
  return FNO_OK;
}

namespace {

// value at x0 of the least-squares line through (x_i, y_i)
double line_at(int n, const double* x, const double* y, double x0) {
  double mx = 0, my = 0;
  for (int i = 0; i < n; ++i) {
    mx += x[i];
    my += y[i];
  }
  mx /= n;
  my /= n;
  double sxy = 0, sxx = 0;
  for (int i = 0; i < n; ++i) {
    sxy += (x[i] - mx) * (y[i] - my);
    sxx += (x[i] - mx) * (x[i] - mx);
  }
  return my + (sxy / sxx) * (x0 - mx);
}

}  // namespace

int fno_xfno(fno_ctx* ctx, int npts, const double* occt, const fno_cc_opts* cc, int kind, const fno_eom_opts* eom,
             int* kept, double* e_cc, double* e_eom, double* e_cc_x, double* e_eom_x) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  auto fail = [&](int st, const std::string& msg) {
    ctx->err = msg;
    return st;
  };
  if (npts < 2 || npts > 16 || !occt || !e_cc || !e_cc_x)
    return fail(FNO_EINVAL, "fno_xfno needs 2..16 thresholds and the e_cc, e_cc_x outputs");
  for (int p = 0; p < npts; ++p) {
    if (!(occt[p] > 0.0 && occt[p] <= 1.0)) return fail(FNO_EINVAL, "occt must lie in (0, 1]");
    for (int q = 0; q < p; ++q)
      if (occt[q] == occt[p]) return fail(FNO_EINVAL, "fno_xfno needs distinct thresholds");
  }
  if (kind != 0 && (kind < FNO_IP || kind > FNO_DEA)) return fail(FNO_EINVAL, "unknown EOM kind");
  fno_eom_opts eo;
  if (eom)
    eo = *eom;
  else
    fno_eom_opts_default(&eo);
  const int nr = kind ? eo.nroots : 0;
  if (kind && (nr < 1 || !e_eom || !e_eom_x)) return fail(FNO_EINVAL, "EOM points need nroots >= 1 and e_eom, e_eom_x");
  int worst = FNO_OK;
  std::vector<double> om(std::max(nr, 1)), et(std::max(nr, 1));
  for (int p = 0; p < npts; ++p) {
    int k = 0;
    int st = fno_truncate(ctx, occt[p], 0, &k, nullptr, nullptr);
    if (st != FNO_OK) return st;
    if (kept) kept[p] = k;
    double ec = 0, etot = 0, rn = 0;
    int it = 0;
    st = fno_ccsdt(ctx, cc, &ec, &etot, &it, &rn);
    if (st == FNO_ENOCONV && kind)
      return fail(FNO_ENOCONV, "fno_xfno: CCSDT did not converge at occt = " + std::to_string(occt[p]));
    if (st != FNO_OK && st != FNO_ENOCONV) return st;
    if (st == FNO_ENOCONV) worst = FNO_ENOCONV;
    e_cc[p] = etot;
    if (kind) {
      st = fno_eom(ctx, (fno_eom_kind)kind, &eo, om.data(), et.data(), nullptr, nullptr);
      if (st != FNO_OK && st != FNO_ENOCONV) return st;
      if (st == FNO_ENOCONV) worst = FNO_ENOCONV;
      for (int r = 0; r < nr; ++r) e_eom[(size_t)p * nr + r] = et[r];
    }
  }
  *e_cc_x = line_at(npts, occt, e_cc, 1.0);
  for (int r = 0; r < nr; ++r) {
    std::vector<double> y(npts);
    for (int p = 0; p < npts; ++p) y[p] = e_eom[(size_t)p * nr + r];
    e_eom_x[r] = line_at(npts, occt, y.data(), 1.0);
  }
  if (worst == FNO_ENOCONV) ctx->err = "fno_xfno: a solve did not converge within max_iter (results written)";
  return worst;
}

int fno_sizes(const fno_ctx* ctx, int* nocc, int* nvir, int* nvir_full) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  if (!ctx->c->loaded) return FNO_ESTATE;
  if (nocc) *nocc = ctx->c->nocc;
  if (nvir) *nvir = ctx->c->nvir;
  if (nvir_full) *nvir_full = ctx->c->nvir_full;
  return FNO_OK;
}

size_t fno_amplitude_size(const fno_ctx* ctx, int block) {
  if (!ctx || !ctx->c || !ctx->c->loaded) return 0;
  long o = ctx->c->nocc, v = ctx->c->nvir;
  if (block == 1) return (size_t)(o * v);
  if (block == 2) return (size_t)(fno::binom_host(o, 2) * fno::binom_host(v, 2));
  if (block == 3) return (size_t)(fno::binom_host(o, 3) * fno::binom_host(v, 3));
  return 0;
}

int fno_get_amplitudes(fno_ctx* ctx, int block, double* buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(buf != nullptr, FNO_EINVAL, "null buffer");
    c.get_amps(block, buf, len);
    return FNO_OK;
  });
}

int fno_set_amplitudes(fno_ctx* ctx, int block, const double* buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(buf != nullptr, FNO_EINVAL, "null buffer");
    c.set_amps(block, buf, len);
    return FNO_OK;
  });
}

int fno_cc_residual(fno_ctx* ctx, fno_prec prec, double* r1, double* r2, double* r3, double* e_corr) {
  return guard(ctx, [&](fno::Context& c) {
    c.cc_residual(to_prec(prec), r1, r2, r3, e_corr);
    return FNO_OK;
  });
}

int fno_get_amplitudes_dev(fno_ctx* ctx, int block, double* d_buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(d_buf != nullptr, FNO_EINVAL, "null buffer");
    c.get_amps(block, d_buf, len, true);
    return FNO_OK;
  });
}

int fno_set_amplitudes_dev(fno_ctx* ctx, int block, const double* d_buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(d_buf != nullptr, FNO_EINVAL, "null buffer");
    c.set_amps(block, d_buf, len, true);
    return FNO_OK;
  });
}

int fno_cc_residual_dev(fno_ctx* ctx, fno_prec prec, double* d_r1, double* d_r2, double* d_r3, double* e_corr) {
  return guard(ctx, [&](fno::Context& c) {
    c.cc_residual(to_prec(prec), d_r1, d_r2, d_r3, e_corr, true);
    return FNO_OK;
  });
}

int fno_eom_sigma_dev(fno_ctx* ctx, fno_eom_kind kind, fno_prec prec, const double* d_r, double* d_sigma,
                      size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(d_r && d_sigma, FNO_EINVAL, "null buffer");
    c.eom_sigma((int)kind, to_prec(prec), d_r, d_sigma, len, true);
    return FNO_OK;
  });
}

size_t fno_eom_size(const fno_ctx* ctx, fno_eom_kind kind) {
  if (!ctx || !ctx->c || !ctx->c->loaded) return 0;
  try {
    return ctx->c->eom_size((int)kind);
  } catch (...) {
    return 0;
  }
}

int fno_eom_sigma(fno_ctx* ctx, fno_eom_kind kind, fno_prec prec, const double* r, double* sigma, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(r && sigma, FNO_EINVAL, "null buffer");
    c.eom_sigma((int)kind, to_prec(prec), r, sigma, len);
    return FNO_OK;
  });
}

int fno_eom_sigma_left(fno_ctx* ctx, fno_eom_kind kind, fno_prec prec, const double* l, double* sigma, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(l && sigma, FNO_EINVAL, "null buffer");
    c.eom_sigma((int)kind, to_prec(prec), l, sigma, len, false, true);
    return FNO_OK;
  });
}

int fno_eom_vectors(fno_ctx* ctx, fno_eom_kind kind, const fno_eom_opts* opts, int left, double* omega,
                    double* vectors, double* res_norm, int* iters) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(kind >= FNO_IP && kind <= FNO_DEA, FNO_EINVAL, "unknown EOM kind");
    FNO_REQUIRE(left == 0 || left == 1, FNO_EINVAL, "left must be 0 (right vectors) or 1 (left vectors)");
    FNO_REQUIRE(c.cc_done, FNO_ESTATE, "fno_eom_vectors needs a converged fno_ccsdt first");
    FNO_REQUIRE(omega != nullptr && vectors != nullptr, FNO_EINVAL, "omega and vectors are required");
    fno::EOMOptions eo = eom_options(opts);
    eo.left = left == 1;
    fno::EOMResult r;
    r.want_vectors = true;
    int st = c.eom((int)kind, eo, r);
    for (int k = 0; k < eo.nroots; ++k) {
      omega[k] = r.omega[k];
      if (res_norm) res_norm[k] = r.res_norm[k];
    }
    std::copy(r.vectors.begin(), r.vectors.end(), vectors);
    if (iters) *iters = r.iters;
    if (st == FNO_ENOCONV) ctx->err = "EOM Davidson did not converge within max_iter";
    return st;
  });
}

int fno_last_flops(const fno_ctx* ctx, double* triples_flops, double* all_flops) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  if (triples_flops) *triples_flops = ctx->c->last_triples_flops;
  if (all_flops) *all_flops = ctx->c->last_all_flops;
  return FNO_OK;
}

int fno_last_trace(const fno_ctx* ctx, double* energies, double* res_norms, int cap, int* n) {
  if (!ctx || !ctx->c || !n) return FNO_EINVAL;
  const auto& c = *ctx->c;
  const int m = (int)c.trace_e.size();
  *n = m;
  for (int k = 0; k < m && k < cap; ++k) {
    if (energies) energies[k] = c.trace_e[k];
    if (res_norms) res_norms[k] = c.trace_r[k];
  }
  return FNO_OK;
}

int fno_profile(fno_ctx* ctx, int on) {
  return guard(ctx, [&](fno::Context& c) {
    c.eng->profile = on != 0;
    return FNO_OK;
  });
}

int fno_profile_filter(fno_ctx* ctx, const char* substr) {
  return guard(ctx, [&](fno::Context& c) {
    c.eng->profile_filter = substr ? std::string(substr) : std::string();
    return FNO_OK;
  });
}

int fno_set_autotune(fno_ctx* ctx, int on) {
  return guard(ctx, [&](fno::Context& c) {
    c.autotune = on != 0;
    c.eng->autotune = c.autotune;
    return FNO_OK;
  });
}

int fno_set_fused(fno_ctx* ctx, int on) {
  return guard(ctx, [&](fno::Context& c) {
    c.fused_r3 = on != 0;
    return FNO_OK;
  });
}

int fno_set_graphs(fno_ctx* ctx, int on) {
  return guard(ctx, [&](fno::Context& c) {
    c.use_graphs = on != 0;
    return FNO_OK;
  });
}

int fno_profile_report(fno_ctx* ctx, char* buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(buf != nullptr, FNO_EINVAL, "null buffer");
    std::string js = c.eng->profile_report();
    FNO_REQUIRE(js.size() + 1 <= len, FNO_EINVAL, "report buffer too small");
    std::memcpy(buf, js.c_str(), js.size() + 1);
    return FNO_OK;
  });
}

size_t fno_debug_tensor_size(fno_ctx* ctx, const char* name) {
  if (!ctx || !ctx->c || !name || !ctx->c->eng->has(name)) return 0;
  return (size_t)ctx->c->eng->get(name)->elems;
}

int fno_debug_tensor(fno_ctx* ctx, const char* name, double* buf, size_t len) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(name && buf && c.eng->has(name), FNO_EINVAL, "unknown tensor");
    fno::Tensor* t = c.eng->get(name);
    FNO_REQUIRE(len == (size_t)t->elems, FNO_EINVAL, "length mismatch");
    FNO_HIP(hipStreamSynchronize(c.eng->stream));
    FNO_HIP(hipMemcpy(buf, t->d, len * sizeof(double), hipMemcpyDeviceToHost));
    return FNO_OK;
  });
}

int fno_debug_gemm(fno_ctx* ctx, fno_prec prec, int tile, long M, long N, long K, int a_kfast, int b_nfast,
                   double alpha, double beta, const double* A, const double* B, double* Cm) {
  return guard(ctx, [&](fno::Context& c) {
    FNO_REQUIRE(A && B && Cm && M > 0 && N > 0 && K >= 0, FNO_EINVAL, "bad GEMM arguments");
    return c.debug_gemm(to_prec(prec), tile, M, N, K, a_kfast != 0, b_nfast != 0, alpha, beta, A, B, Cm);
  });
}


long fno_mlp_num_params(void) { return (long)fno::Mlp::num_params(); }

int fno_mlp_create(int hip_device, fno_mlp** out) {
  if (!out) return FNO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return FNO_EDEVICE;
  try {
    auto* h = new fno_mlp;
    h->m = new fno::Mlp(hip_device);
    *out = h;
    return FNO_OK;
  } catch (const fno::Error& e) {
    return e.code;
  } catch (...) {
    return FNO_EDEVICE;
  }
}

void fno_mlp_destroy(fno_mlp* h) {
  if (!h) return;
  delete h->m;
  delete h;
}

const char* fno_mlp_last_error(const fno_mlp* h) { return h ? h->err.c_str() : "null network handle"; }

long fno_mlp_samples(const fno_mlp* h) { return (h && h->m) ? (long)h->m->samples() : 0; }

int fno_mlp_collect(fno_mlp* h, fno_ctx* ctx, long max_samples) {
  if (!h || !h->m) return FNO_EINVAL;
  return guard(ctx, [&](fno::Context& c) {
    c.ml_collect(*h->m, (int64_t)max_samples);
    return FNO_OK;
  });
}

int fno_mlp_train(fno_mlp* h, int steps, int batch, double lr, unsigned long seed, double* loss) {
  return mguard(h, [&](fno::Mlp& m) {
    const double l = m.train(steps, batch, lr, (uint64_t)seed);
    if (loss) *loss = l;
    return FNO_OK;
  });
}

int fno_mlp_save(fno_mlp* h, const char* path) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(path != nullptr, FNO_EINVAL, "null path");
    m.save(path);
    return FNO_OK;
  });
}

int fno_mlp_load(fno_mlp* h, const char* path) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(path != nullptr, FNO_EINVAL, "null path");
    m.load(path);
    return FNO_OK;
  });
}

int fno_mlp_params(fno_mlp* h, float* buf, size_t len, int set) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(buf != nullptr && len == (size_t)fno::Mlp::num_params(), FNO_EINVAL,
                "buffer must hold fno_mlp_num_params() floats");
    if (set)
      m.set_params(buf);
    else
      m.get_params(buf);
    return FNO_OK;
  });
}

int fno_mlp_loss_grad(fno_mlp* h, const float* X, const float* T, long B, float* grad, double* loss) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(X && T && grad && B > 0, FNO_EINVAL, "bad arguments");
    float *dX = nullptr, *dT = nullptr;
    FNO_HIP(hipMalloc(&dX, (size_t)B * fno::Mlp::F * sizeof(float)));
    FNO_HIP(hipMalloc(&dT, (size_t)B * fno::Mlp::O * sizeof(float)));
    FNO_HIP(hipMemcpy(dX, X, (size_t)B * fno::Mlp::F * sizeof(float), hipMemcpyHostToDevice));
    FNO_HIP(hipMemcpy(dT, T, (size_t)B * fno::Mlp::O * sizeof(float), hipMemcpyHostToDevice));
    const double l = m.loss_grad(dX, dT, B);
    FNO_HIP(hipMemcpy(grad, m.grad(), (size_t)fno::Mlp::num_params() * sizeof(float), hipMemcpyDeviceToHost));
    (void)hipFree(dX);
    (void)hipFree(dT);
    if (loss) *loss = l;
    return FNO_OK;
  });
}

int fno_mlp_predict(fno_mlp* h, const float* X, long n, float* Y) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(X && Y && n > 0, FNO_EINVAL, "bad arguments");
    float *dX = nullptr, *dY = nullptr;
    FNO_HIP(hipMalloc(&dX, (size_t)n * fno::Mlp::F * sizeof(float)));
    FNO_HIP(hipMalloc(&dY, (size_t)n * fno::Mlp::O * sizeof(float)));
    FNO_HIP(hipMemcpy(dX, X, (size_t)n * fno::Mlp::F * sizeof(float), hipMemcpyHostToDevice));
    m.predict_bf16(dX, n, dY, m.stream);
    FNO_HIP(hipStreamSynchronize(m.stream));
    FNO_HIP(hipMemcpy(Y, dY, (size_t)n * fno::Mlp::O * sizeof(float), hipMemcpyDeviceToHost));
    (void)hipFree(dX);
    (void)hipFree(dY);
    return FNO_OK;
  });
}

int fno_mlp_dataset(fno_mlp* h, float* X, float* T, long n) {
  return mguard(h, [&](fno::Mlp& m) {
    FNO_REQUIRE(X && T, FNO_EINVAL, "null buffers");
    m.read_samples(X, T, (int64_t)n);
    return FNO_OK;
  });
}

int fno_set_guess_model(fno_ctx* ctx, fno_mlp* h) {
  return guard(ctx, [&](fno::Context& c) {
    if (h) FNO_REQUIRE(h->m && h->m->device == c.device, FNO_EINVAL, "the network lives on another device");
    c.guess_model = h ? h->m : nullptr;
    return FNO_OK;
  });
}

int fno_last_guess_accepted(const fno_ctx* ctx) {
  if (!ctx || !ctx->c) return FNO_EINVAL;
  return ctx->c->last_guess_accepted ? 1 : 0;
}
}  // extern "C"

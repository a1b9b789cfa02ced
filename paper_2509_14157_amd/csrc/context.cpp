// Context lifetime, Hamiltonian loading and the FNO front end (Section 1.2).
#include "context.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "eom_space.hpp"
#include "linalg.hpp"

namespace fno {

Context::Context(int dev) : device(dev) {
  int ndev = 0;
  FNO_HIP(hipGetDeviceCount(&ndev));
  FNO_REQUIRE(dev >= 0 && dev < ndev, kEDEVICE, "no such HIP device");
  hipDeviceProp_t prop;
  FNO_HIP(hipGetDeviceProperties(&prop, dev));
  FNO_REQUIRE(std::string(prop.gcnArchName).rfind("gfx950", 0) == 0, kEDEVICE,
              std::string("library built for gfx950, device is ") + prop.gcnArchName);
  eng = std::make_unique<Engine>(dev);
}

void Context::set_stream(hipStream_t s) {
  FNO_HIP(hipDeviceSynchronize());
  user_stream = s;
  eng->stream = s ? s : eng->own_stream();
  // recordings remember the stream they were last launched on
  cc_prog_.clear();
  if (eom_) {
    eom_->rg.prog.clear();
    eom_->lg.prog.clear();
  }
}

void Context::reset_engine(std::unique_ptr<Engine> e) {
  FNO_HIP(hipDeviceSynchronize());
  cc_prog_.clear();  // recorded launches point into the old engine
  cc_stable_ = false;
  eom_.reset();
  eng = std::move(e);
  if (user_stream) eng->stream = user_stream;
  eng->autotune = autotune;
}

Context::~Context() {
  (void)hipSetDevice(device);
  (void)hipDeviceSynchronize();
  for (double* p : owned_) (void)hipFree(p);
  if (host_pin_) (void)hipHostFree(host_pin_);
  if (e_ready_) (void)hipEventDestroy(e_ready_);
  eng.reset();
}

void Context::load(int o, int v, const double* f, const double* g, double en) {
  FNO_REQUIRE(o >= 1 && v >= 1 && o + v <= 256, kEINVAL, "need 1 <= nocc, nvir and nocc + nvir <= 256");
  FNO_REQUIRE(f && g, kEINVAL, "null input array");
  FNO_REQUIRE(std::isfinite(en), kENONFINITE, "non-finite e_nuc");
  const int n = o + v;
  const int64_t n2 = (int64_t)n * n, n4 = n2 * n2;
  double fmax = 0, gmax = 0;
  for (int64_t i = 0; i < n2; ++i) {
    FNO_REQUIRE(std::isfinite(f[i]), kENONFINITE, "non-finite Fock element");
    fmax = std::max(fmax, std::fabs(f[i]));
  }
  for (int64_t i = 0; i < n4; ++i) {
    FNO_REQUIRE(std::isfinite(g[i]), kENONFINITE, "non-finite integral");
    gmax = std::max(gmax, std::fabs(g[i]));
  }
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      FNO_REQUIRE(std::fabs(f[(size_t)p * n + q] - f[(size_t)q * n + p]) <= 1e-10 * std::max(1.0, fmax), kEINVAL,
                  "Fock matrix is not symmetric");
      if (p < o && q >= o) FNO_REQUIRE(std::fabs(f[(size_t)p * n + q]) < 1e-10, kEINVAL, "f_ov must vanish");
    }
  const double tol = 1e-10 * std::max(1.0, gmax);
  auto G = [&](int p, int q, int r, int s) { return g[(((int64_t)p * n + q) * n + r) * n + s]; };
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s) {
          double x = G(p, q, r, s);
          if (std::fabs(x + G(q, p, r, s)) > tol || std::fabs(x + G(p, q, s, r)) > tol ||
              std::fabs(x - G(r, s, p, q)) > tol)
            throw Error(kEINVAL, "integrals lack <pq||rs> = -<qp||rs> = -<pq||sr> = <rs||pq> symmetry");
        }
  // reset any previous problem
  if (loaded) {
    reset_engine(std::make_unique<Engine>(device));
    for (double* p : owned_) (void)hipFree(p);
    owned_.clear();
    eom_.reset();
  }
  nocc = o;
  nvir = nvir_full = v;
  e_nuc = en;
  fock_full.assign(f, f + n2);
  fock = fock_full;
  Engine& e = *eng;
  SpaceSizes full;
  full.n = {{'N', n}};
  Tensor* Gf = e.create("Gfull", "N,N,N,N", full);
  e.set_sym(Gf, {{0, 1}, {2, 3}});
  FNO_HIP(hipMemcpy(Gf->d, g, (size_t)n4 * sizeof(double), hipMemcpyHostToDevice));
  // E_ref = sum_i f_ii - 1/2 sum_ij <ij||ij>
  double er = 0;
  for (int i = 0; i < o; ++i) er += f[(size_t)i * n + i];
  for (int i = 0; i < o; ++i)
    for (int j = 0; j < o; ++j) er -= 0.5 * G(i, j, i, j);
  e_ref = er + en;
  loaded = true;
  truncated = false;
  cc_ready = cc_done = false;
  // working space = full space until fno_truncate is called
  SpaceSizes ws;
  ws.n = {{'n', n}};
  Tensor* Gw = e.create("G", "n,n,n,n", ws);
  launch_axpby(Gw->d, Gf->d, 1.0, 0.0, n4, e.stream);
  Tensor* F0 = e.create("F0", "n,n", ws);
  FNO_HIP(hipMemcpy(F0->d, f, (size_t)n2 * sizeof(double), hipMemcpyHostToDevice));
  // core Hamiltonian h = f - sum_i <pi||qi> (host; n^3)
  std::vector<double> h(n2);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double s = f[(size_t)p * n + q];
      for (int i = 0; i < o; ++i) s -= G(p, i, q, i);
      h[(size_t)p * n + q] = s;
    }
  Tensor* H = e.create("Hcore", "n,n", ws);
  FNO_HIP(hipMemcpy(H->d, h.data(), (size_t)n2 * sizeof(double), hipMemcpyHostToDevice));
  FNO_HIP(hipDeviceSynchronize());
}

int Context::debug_gemm(Prec p, int tile, int64_t M, int64_t N, int64_t K, bool a_kfast, bool b_nfast,
                        double alpha, double beta, const double* A, const double* B, double* Cm) {
  // operands are converted on the host to the GEMM input type
  auto to_bf16 = [](float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    uint32_t r = ((u >> 16) & 1u) + 0x7fffu;  // round to nearest even
    return (uint16_t)((u + r) >> 16);
  };
  auto from_bf16 = [](uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
  };
  const int64_t na = M * K, nb = K * N, nc = M * N;
  void *dA = nullptr, *dB = nullptr, *dAl = nullptr, *dBl = nullptr, *dC = nullptr;
  std::vector<char> hA, hB, hAl, hBl, hC;
  auto conv = [&](const double* src, int64_t n, std::vector<char>& hi, std::vector<char>& lo) {
    if (p == Prec::FP64) {
      hi.assign((const char*)src, (const char*)(src + n));
    } else if (p == Prec::FP32) {
      hi.resize(n * 4);
      for (int64_t i = 0; i < n; ++i) ((float*)hi.data())[i] = (float)src[i];
    } else {
      hi.resize(n * 2);
      lo.resize(n * 2);
      for (int64_t i = 0; i < n; ++i) {
        float x = (float)src[i];
        uint16_t h = to_bf16(x);
        ((uint16_t*)hi.data())[i] = h;
        ((uint16_t*)lo.data())[i] = to_bf16(x - from_bf16(h));
      }
    }
  };
  conv(A, na, hA, hAl);
  conv(B, nb, hB, hBl);
  if (p == Prec::FP64) {
    hC.assign((const char*)Cm, (const char*)(Cm + nc));
  } else {
    hC.resize(nc * 4);
    for (int64_t i = 0; i < nc; ++i) ((float*)hC.data())[i] = (float)Cm[i];
  }
  auto up = [&](std::vector<char>& h, void** d) {
    if (h.empty()) return;
    FNO_HIP(hipMalloc(d, h.size()));
    FNO_HIP(hipMemcpy(*d, h.data(), h.size(), hipMemcpyHostToDevice));
  };
  up(hA, &dA);
  up(hB, &dB);
  up(hAl, &dAl);
  up(hBl, &dBl);
  up(hC, &dC);
  GemmArgs g{};
  g.prec = p;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = dA;
  g.A_lo = dAl;
  g.lda = a_kfast ? K : M;
  g.a_kfast = a_kfast;
  g.B = dB;
  g.B_lo = dBl;
  g.ldb = b_nfast ? N : K;
  g.b_nfast = b_nfast;
  g.C = dC;
  g.ldc = N;
  g.alpha = alpha;
  g.beta = beta;
  g.tile = tile;
  g.split = gemm_split_factor(g);
  void* dW = nullptr;
  if (g.split > 1) {
    FNO_HIP(hipMalloc(&dW, gemm_split_bytes(g, g.split)));
    g.ws = dW;
  }
  launch_gemm(g, eng->stream);
  FNO_HIP(hipStreamSynchronize(eng->stream));
  if (dW) FNO_HIP(hipFree(dW));
  FNO_HIP(hipMemcpy(hC.data(), dC, hC.size(), hipMemcpyDeviceToHost));
  if (p == Prec::FP64)
    std::memcpy(Cm, hC.data(), nc * 8);
  else
    for (int64_t i = 0; i < nc; ++i) Cm[i] = ((float*)hC.data())[i];
  for (void* d : {dA, dB, dAl, dBl, dC})
    if (d) FNO_HIP(hipFree(d));
  return kOK;
}

static void fix_signs(int rows, int cols, std::vector<double>& U) {
  for (int j = 0; j < cols; ++j) {
    int best = 0;
    for (int i = 1; i < rows; ++i)
      if (std::fabs(U[(size_t)i * cols + j]) > std::fabs(U[(size_t)best * cols + j])) best = i;
    if (U[(size_t)best * cols + j] < 0)
      for (int i = 0; i < rows; ++i) U[(size_t)i * cols + j] = -U[(size_t)i * cols + j];
  }
}

void Context::truncate(double occt, int keep, int* kept, double* emp2, double* occ_out) {
  FNO_REQUIRE(loaded, kESTATE, "no Hamiltonian loaded");
  FNO_REQUIRE(keep > 0 || (occt > 0.0 && occt <= 1.0), kEINVAL, "occt must lie in (0, 1]");
  FNO_REQUIRE(keep <= nvir_full, kEINVAL, "nvir_keep exceeds the virtual space");
  Engine& e = *eng;
  const int o = nocc, V = nvir_full, N = o + V;
  // drop the previous working space
  if (cc_ready || truncated || e.has("G")) {
    FNO_HIP(hipDeviceSynchronize());
    Tensor* Gf = e.get("Gfull");
    std::vector<double> hostg;  // not needed: the full integrals stay on the device
    (void)Gf;
    auto ge = std::make_unique<Engine>(device);
    // move the full integrals into a fresh engine (everything else is rebuilt)
    SpaceSizes full;
    full.n = {{'N', N}};
    Tensor* nf = ge->create("Gfull", "N,N,N,N", full);
    ge->set_sym(nf, {{0, 1}, {2, 3}});
    FNO_HIP(hipMemcpy(nf->d, Gf->d, (size_t)Gf->elems * sizeof(double), hipMemcpyDeviceToDevice));
    for (double* p : owned_) (void)hipFree(p);
    owned_.clear();
    eom_.reset();
    reset_engine(std::move(ge));
    cc_ready = cc_done = false;
  }
  Engine& E = *eng;
  SpaceSizes full;
  full.n = {{'o', o}, {'v', V}, {'N', N}};
  // MP2 amplitudes t_ij^ab = <ab||ij> / e_ij^ab  (eqs 8-9)
  E.view("Gf_vvoo", E.get("Gfull"), {{o, V}, {o, V}, {0, o}, {0, o}});
  E.view("Gf_oovv", E.get("Gfull"), {{0, o}, {0, o}, {o, V}, {o, V}});
  Tensor* num = E.create("MP2num", "oo,vv", full);
  Tensor* t2 = E.create("MP2t", "oo,vv", full);
  Tensor* den = E.create("MP2den", "oo,vv", full);
  E.create("Dvv", "v,v", full);
  E.create("Emp2", "", full);
  E.term("MP2num[ijab] += 1 * Gf_vvoo[abij]");
  std::vector<double> eo(o), ev(V);
  for (int i = 0; i < o; ++i) eo[i] = fock_full[(size_t)i * N + i];
  for (int a = 0; a < V; ++a) ev[a] = fock_full[(size_t)(o + a) * N + (o + a)];
  double* d_e = alloc(o + V);
  FNO_HIP(hipMemcpy(d_e, eo.data(), o * sizeof(double), hipMemcpyHostToDevice));
  FNO_HIP(hipMemcpy(d_e + o, ev.data(), V * sizeof(double), hipMemcpyHostToDevice));
  MatDim md{};
  md.ngroups = 2;
  md.grp[0] = {2, o, (int64_t)binom_host(o, 2), {0, 1}};
  md.grp[1] = {2, V, (int64_t)binom_host(V, 2), {2, 3}};
  md.size = md.grp[0].count * md.grp[1].count;
  launch_denominators(E.tables, md, 2, d_e, d_e + o, den->d, E.stream);
  launch_jacobi(t2->d, num->d, den->d, nullptr, md.size, E.stream);
  // E_MP2 = 1/4 sum <ij||ab> t_ij^ab
  E.term("Emp2[] += 0.25 * Gf_oovv[ijab] * MP2t[ijab]");
  // D_ab = 1/2 sum_{cij} t_ij^ac t_ij^bc  (eq 10 with t from eq 8)
  E.term("Dvv[ab] += 0.5 * MP2t[ijac] * MP2t[ijbc]");
  std::vector<double> D((size_t)V * V);
  double em;
  FNO_HIP(hipMemcpy(D.data(), E.get("Dvv")->d, D.size() * sizeof(double), hipMemcpyDeviceToHost));
  FNO_HIP(hipMemcpy(&em, E.get("Emp2")->d, sizeof(double), hipMemcpyDeviceToHost));
  e_mp2_full = em;
  for (int a = 0; a < V; ++a)
    for (int b = 0; b < a; ++b) {
      double s = 0.5 * (D[(size_t)a * V + b] + D[(size_t)b * V + a]);
      D[(size_t)a * V + b] = D[(size_t)b * V + a] = s;
    }
  std::vector<double> w, U;
  sym_eig(V, D, w, U);
  // descending occupation
  std::vector<double> occ(V), Ud((size_t)V * V);
  for (int j = 0; j < V; ++j) {
    occ[j] = w[V - 1 - j];
    for (int i = 0; i < V; ++i) Ud[(size_t)i * V + j] = U[(size_t)i * V + (V - 1 - j)];
  }
  fix_signs(V, V, Ud);
  int k = keep;
  if (k <= 0) {
    if (occt >= 1.0) {
      k = V;
    } else {
      double total = std::accumulate(occ.begin(), occ.end(), 0.0);
      double target = occt * total * (1.0 - 1e-12), cs = 0;
      k = V;
      for (int j = 0; j < V; ++j) {
        cs += occ[j];
        if (cs >= target) {
          k = j + 1;
          break;
        }
      }
      while (k < V && std::fabs(occ[k - 1] - occ[k]) <= 1e-10 * std::fabs(occ[k - 1])) ++k;
    }
  }
  // semicanonicalise the kept block: f' = Uk^T f_vv Uk
  std::vector<double> fk((size_t)k * k, 0.0);
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      double s = 0;
      for (int c = 0; c < V; ++c)
        for (int d = 0; d < V; ++d)
          s += Ud[(size_t)c * V + a] * fock_full[(size_t)(o + c) * N + (o + d)] * Ud[(size_t)d * V + b];
      fk[(size_t)a * k + b] = s;
    }
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < a; ++b) fk[(size_t)a * k + b] = fk[(size_t)b * k + a] = 0.5 * (fk[(size_t)a * k + b] + fk[(size_t)b * k + a]);
  std::vector<double> ws, Vs;
  sym_eig(k, fk, ws, Vs);
  fix_signs(k, k, Vs);
  // full transformation C (N x n): diag(1_o, Uk Vs)
  const int n = o + k;
  std::vector<double> C((size_t)N * n, 0.0);
  for (int i = 0; i < o; ++i) C[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < V; ++c)
    for (int b = 0; b < k; ++b) {
      double s = 0;
      for (int a = 0; a < k; ++a) s += Ud[(size_t)c * V + a] * Vs[(size_t)a * k + b];
      C[(size_t)(o + c) * n + (o + b)] = s;
    }
  // transformed Fock (host) and integrals (device, four rotations)
  std::vector<double> f2((size_t)n * n, 0.0);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double s = 0;
      for (int r = 0; r < N; ++r) {
        double cr = C[(size_t)r * n + p];
        if (cr == 0) continue;
        for (int t = 0; t < N; ++t) s += cr * fock_full[(size_t)r * N + t] * C[(size_t)t * n + q];
      }
      f2[(size_t)p * n + q] = s;
    }
  for (int a = o; a < n; ++a)
    for (int b = o; b < n; ++b)
      if (a != b) f2[(size_t)a * n + b] = 0.0;  // exactly diagonal after semicanonicalisation
  full.n['n'] = n;
  Tensor* Cf = E.create("Cf", "N,n", full);
  FNO_HIP(hipMemcpy(Cf->d, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
  // rotation buffers
  E.create("Rot1", "N,N,N,n", full);
  E.term("Rot1[qrsP] += 1 * Gfull[pqrs] * Cf[pP]");
  E.create("Rot2", "N,N,n,n", full);
  E.term("Rot2[rsPQ] += 1 * Rot1[qrsP] * Cf[qQ]");
  E.drop("Rot1");
  E.create("Rot3", "N,n,n,n", full);
  E.term("Rot3[sPQR] += 1 * Rot2[rsPQ] * Cf[rR]");
  E.drop("Rot2");
  SpaceSizes wsz;
  wsz.n = {{'n', n}};
  Tensor* Gw = E.create("G", "n,n,n,n", wsz);
  E.term("G[PQRS] += 1 * Rot3[sPQR] * Cf[sS]");
  E.set_sym(Gw, {{0, 1}, {2, 3}});  // <PQ||RS>: antisymmetric slot pairs
  E.drop("Rot3");
  for (const char* nm : {"MP2num", "MP2t", "MP2den", "Dvv", "Emp2", "Cf", "Gf_vvoo", "Gf_oovv"}) E.drop(nm);
  (void)Gw;
  fock = f2;
  nvir = k;
  Tensor* F0 = E.create("F0", "n,n", wsz);
  FNO_HIP(hipMemcpy(F0->d, f2.data(), f2.size() * sizeof(double), hipMemcpyHostToDevice));
  // core Hamiltonian h = f - sum_i <pi||qi> from the transformed integrals
  std::vector<double> gtr((size_t)n * o * n * o);
  {
    E.create("Gtr", "n,o,n,o", SpaceSizes{{{'n', n}, {'o', o}}});
    E.view("G_nono", E.get("G"), {{0, n}, {0, o}, {0, n}, {0, o}});
    E.term("Gtr[piqj] += 1 * G_nono[piqj]");
    FNO_HIP(hipMemcpy(gtr.data(), E.get("Gtr")->d, gtr.size() * sizeof(double), hipMemcpyDeviceToHost));
    E.drop("Gtr");
    E.drop("G_nono");
  }
  std::vector<double> h((size_t)n * n);
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double s = f2[(size_t)p * n + q];
      for (int i = 0; i < o; ++i) s -= gtr[(((size_t)p * o + i) * n + q) * o + i];
      h[(size_t)p * n + q] = s;
    }
  Tensor* H = E.create("Hcore", "n,n", wsz);
  FNO_HIP(hipMemcpy(H->d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  // E_MP2 in the truncated space: the same formula over the kept
  // semicanonical virtuals (their orbital energies the diagonal of f2)
  {
    SpaceSizes tsz;
    tsz.n = {{'o', o}, {'v', k}};
    E.view("Gt_vvoo", E.get("G"), {{o, k}, {o, k}, {0, o}, {0, o}});
    E.view("Gt_oovv", E.get("G"), {{0, o}, {0, o}, {o, k}, {o, k}});
    Tensor* tnum = E.create("MP2tnum", "oo,vv", tsz);
    Tensor* tamp = E.create("MP2tamp", "oo,vv", tsz);
    Tensor* tden = E.create("MP2tden", "oo,vv", tsz);
    E.create("Emp2t", "", tsz);
    E.term("MP2tnum[ijab] += 1 * Gt_vvoo[abij]");
    std::vector<double> et(o + k);
    for (int i = 0; i < o; ++i) et[i] = eo[i];
    for (int a = 0; a < k; ++a) et[o + a] = f2[(size_t)(o + a) * n + (o + a)];
    double* d_et = alloc(o + k);
    FNO_HIP(hipMemcpy(d_et, et.data(), et.size() * sizeof(double), hipMemcpyHostToDevice));
    MatDim mt{};
    mt.ngroups = 2;
    mt.grp[0] = {2, o, (int64_t)binom_host(o, 2), {0, 1}};
    mt.grp[1] = {2, k, (int64_t)binom_host(k, 2), {2, 3}};
    mt.size = mt.grp[0].count * mt.grp[1].count;
    launch_denominators(E.tables, mt, 2, d_et, d_et + o, tden->d, E.stream);
    launch_jacobi(tamp->d, tnum->d, tden->d, nullptr, mt.size, E.stream);
    E.term("Emp2t[] += 0.25 * Gt_oovv[ijab] * MP2tamp[ijab]");
    FNO_HIP(hipMemcpy(&e_mp2_trunc, E.get("Emp2t")->d, sizeof(double), hipMemcpyDeviceToHost));
    for (const char* nm : {"MP2tnum", "MP2tamp", "MP2tden", "Emp2t", "Gt_vvoo", "Gt_oovv"}) E.drop(nm);
  }
  FNO_HIP(hipDeviceSynchronize());
  // E_ref is unchanged: the occupied block is not rotated
  truncated = true;
  if (kept) *kept = k;
  if (emp2) *emp2 = em;
  if (occ_out) std::copy(occ.begin(), occ.end(), occ_out);
}

}  // namespace fno

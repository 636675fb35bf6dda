// Drives every entry point of the C ABI once, through its success path and
// its argument checks, from a program built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side of the library (host.hip) and
// on this file.  It checks statuses and a few properties of the results
// (finite, symmetric, repeatable in the deterministic mode, ENOMEM under a
// workspace cap); the numerical parity of each call is the Python suite's
// job.  The sanitizers report any out-of-bounds access, use after free or
// undefined operation in the host code and abort the program.
// Exit status 0 = every check passed.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mderi.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAIL: %s (last error: %s)\n", what, mderi_last_error());
    ++failures;
  } else {
    std::printf("ok: %s\n", what);
  }
  std::fflush(stdout);
}

// Small deterministic generator (64-bit LCG, top 53 bits).
struct Lcg {
  unsigned long long s;
  double uniform() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * 0x1p-53;
  }
};

struct Shells {
  std::vector<int> l, K;
  std::vector<double> exps, coefs, centers;
  int nao() const {
    int n = 0;
    for (int x : l) n += 2 * x + 1;
    return n;
  }
};

Shells make_shells(const std::vector<int> &l, const std::vector<int> &K, double box, double lo, double hi,
                   unsigned long long seed) {
  Lcg g{seed};
  Shells s;
  s.l = l;
  s.K = K;
  for (size_t i = 0; i < l.size(); ++i) {
    for (int k = 0; k < 3; ++k) s.centers.push_back(box * g.uniform());
    for (int p = 0; p < K[i]; ++p) {
      s.exps.push_back(std::exp(std::log(lo) + (std::log(hi) - std::log(lo)) * g.uniform()));
      s.coefs.push_back(K[i] > 1 ? 0.1 + 0.9 * g.uniform() : 1.0);
    }
  }
  return s;
}

mderi_basis_t upload(mderi_ctx_t c, const Shells &s) {
  mderi_basis_t b = nullptr;
  const mderi_status st = mderi_basis_upload(c, (int)s.l.size(), s.l.data(), s.K.data(), s.exps.data(),
                                             s.coefs.data(), s.centers.data(), nullptr, 1, &b);
  expect(st == MDERI_OK && b, "mderi_basis_upload");
  return b;
}

double *dev(size_t n) {
  void *p = nullptr;
  if (hipMalloc(&p, sizeof(double) * (n ? n : 1)) != hipSuccess) {
    std::fprintf(stderr, "hipMalloc failed\n");
    std::exit(2);
  }
  return (double *)p;
}

std::vector<double> host(const double *d, size_t n) {
  std::vector<double> h(n);
  if (hipMemcpy(h.data(), d, sizeof(double) * n, hipMemcpyDeviceToHost) != hipSuccess) {
    std::fprintf(stderr, "hipMemcpy failed\n");
    std::exit(2);
  }
  return h;
}

bool all_finite(const std::vector<double> &v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

bool symmetric(const std::vector<double> &m, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j)
      if (m[(size_t)i * n + j] != m[(size_t)j * n + i]) return false;
  return true;
}

}  // namespace

int main() {
  // argument checks that need no device
  expect(mderi_create(0, nullptr) == MDERI_EINVAL, "create rejects a NULL handle pointer");
  expect(mderi_eri4(nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, 0, nullptr, nullptr) == MDERI_EINVAL,
         "eri4 rejects a NULL context");
  expect(std::strlen(mderi_last_error()) > 0, "last_error describes the failure");
  mderi_destroy(nullptr);
  mderi_basis_free(nullptr);

  mderi_ctx_t c = nullptr;
  if (mderi_create(0, &c) != MDERI_OK) {
    std::fprintf(stderr, "mderi_create failed: %s\n", mderi_last_error());
    return 2;
  }
  const Shells s = make_shells({0, 1, 2, 1, 3, 0, 2}, {2, 1, 1, 2, 1, 3, 2}, 3.0, 0.1, 30.0, 11);
  const Shells ax = make_shells({0, 1, 2, 0, 1, 2, 3, 3}, {1, 1, 1, 1, 1, 1, 1, 1}, 3.0, 0.2, 8.0, 12);
  mderi_basis_t b = upload(c, s), a = upload(c, ax);
  const int nao = s.nao(), nsh = (int)s.l.size();
  expect(mderi_basis_nao(b) == nao && mderi_basis_nshell(b) == nsh, "basis sizes");
  {
    const int bad_l[1] = {MDERI_LMAX + 1}, one[1] = {1};
    const double e[1] = {1.0}, co[1] = {1.0}, ce[3] = {0, 0, 0};
    mderi_basis_t x = nullptr;
    expect(mderi_basis_upload(c, 1, bad_l, one, e, co, ce, nullptr, 1, &x) == MDERI_EUNSUPPORTED,
           "upload rejects l beyond the maximum");
  }

  // 4-centre class batch: (d d | p p), plus its checks
  const int32_t bra[4] = {2, 2, 6, 2}, ket[4] = {1, 3, 3, 3};
  const size_t nv = 2 * 25 * 9 * 2;
  double *V = dev(nv);
  expect(mderi_eri4(c, b, 2, bra, 2, ket, V, nv, nullptr, nullptr) == MDERI_OK, "eri4");
  const std::vector<double> v1 = host(V, nv);
  expect(all_finite(v1), "eri4 output finite");
  expect(mderi_eri4(c, b, 2, bra, 2, ket, V, nv - 1, nullptr, nullptr) == MDERI_ESIZE, "eri4 short output");
  const int32_t mixed[4] = {2, 2, 1, 3};
  expect(mderi_eri4(c, b, 2, mixed, 2, ket, V, nv, nullptr, nullptr) == MDERI_EINVAL, "eri4 mixed classes");
  const int32_t oob[2] = {0, nsh};
  expect(mderi_eri4(c, b, 1, oob, 2, ket, V, nv, nullptr, nullptr) == MDERI_EINVAL, "eri4 shell out of range");
  int nvar = -1;
  expect(mderi_eri4_tile_variants(c, b, 2, bra, 2, ket, &nvar) == MDERI_OK && nvar >= 0, "eri4_tile_variants");
  {
    mderi_opts o{};
    o.flags = MDERI_FLAG_AUTOTUNE;
    expect(mderi_eri4(c, b, 2, bra, 2, ket, V, nv, &o, nullptr) == MDERI_OK, "eri4 autotuned");
    const std::vector<double> v2 = host(V, nv);
    double d = 0.0, m = 0.0;
    for (size_t i = 0; i < nv; ++i) {
      d = std::fmax(d, std::fabs(v2[i] - v1[i]));
      m = std::fmax(m, std::fabs(v1[i]));
    }
    expect(d <= 1e-12 * m, "eri4 autotuned agrees");
  }
  expect(mderi_eri4_noalloc(c, b, 2, bra, 2, ket, V, nv, nullptr, nullptr) == MDERI_OK, "eri4_noalloc");
  {
    // the same integrals; the work split may differ from the one v1 took (the
    // autotuner's choice is kept in the context), hence the order of sums
    const std::vector<double> v3 = host(V, nv);
    double d = 0.0, m = 0.0;
    for (size_t i = 0; i < nv; ++i) {
      d = std::fmax(d, std::fabs(v3[i] - v1[i]));
      m = std::fmax(m, std::fabs(v1[i]));
    }
    expect(d <= 1e-12 * m, "eri4_noalloc agrees with eri4");
  }

  // Schwarz factors of every canonical pair
  std::vector<int32_t> pairs;
  for (int i = 0; i < nsh; ++i)
    for (int j = 0; j <= i; ++j) {
      pairs.push_back(i);
      pairs.push_back(j);
    }
  const int np = (int)pairs.size() / 2;
  double *Q = dev(np);
  expect(mderi_schwarz(c, b, np, pairs.data(), Q, nullptr) == MDERI_OK, "schwarz");
  expect(all_finite(host(Q, np)), "schwarz finite");

  // 3-centre: one class, and the task list over every pair and aux shell
  const int32_t ppair[4] = {2, 1, 6, 3}, paux[2] = {2, 5};
  const size_t n3 = 2 * 15 * 5 * 2;
  double *V3 = dev(n3);
  expect(mderi_eri3(c, b, a, 2, ppair, 2, paux, V3, n3, nullptr, nullptr) == MDERI_OK, "eri3");
  expect(all_finite(host(V3, n3)), "eri3 finite");
  std::vector<int32_t> all_aux(ax.l.size());
  for (size_t k = 0; k < all_aux.size(); ++k) all_aux[k] = (int32_t)k;
  size_t nrow = 0, ncol = 0;
  for (int p = 0; p < np; ++p) nrow += (size_t)(2 * s.l[pairs[2 * p]] + 1) * (2 * s.l[pairs[2 * p + 1]] + 1);
  for (int x : ax.l) ncol += 2 * x + 1;
  double *B = dev(nrow * ncol);
  for (int rep = 0; rep < 2; ++rep) {
    mderi_opts o{};
    o.flags = MDERI_FLAG_GRAPH;
    expect(mderi_eri3_batch(c, b, a, np, pairs.data(), (int)all_aux.size(), all_aux.data(), B, nrow * ncol, &o,
                            nullptr) == MDERI_OK,
           rep ? "eri3_batch graph replay" : "eri3_batch graph capture");
  }
  expect(all_finite(host(B, nrow * ncol)), "eri3_batch finite");

  // 2-centre metric block and density-fitted J
  const int32_t sa[2] = {3, 6}, sc[1] = {6};
  double *V2 = dev(2 * 25 * 25);
  const int32_t dsh[2] = {2, 5}, dsh2[2] = {2, 5};
  expect(mderi_eri2(c, a, 2, dsh, 2, dsh2, V2, 2 * 25 * 2, nullptr, nullptr) == MDERI_OK, "eri2");
  expect(mderi_eri2(c, a, 2, sa, 1, sc, V2, 2 * 25 * 25, nullptr, nullptr) == MDERI_EINVAL, "eri2 mixed l");

  // density, J and K in both accumulation modes, energies, gradient
  std::vector<double> Dh((size_t)nao * nao);
  {
    Lcg g{5};
    std::vector<double> C((size_t)nao * 3);
    for (double &x : C) x = g.uniform() - 0.5;
    for (int i = 0; i < nao; ++i)
      for (int j = 0; j < nao; ++j) {
        double t = 0.0;
        for (int k = 0; k < 3; ++k) t += C[(size_t)i * 3 + k] * C[(size_t)j * 3 + k];
        Dh[(size_t)i * nao + j] = t;
      }
  }
  const size_t nn = (size_t)nao * nao;
  double *D = dev(nn), *J = dev(nn), *K = dev(nn), *E = dev(2), *J2 = dev(nn), *K2 = dev(nn);
  (void)hipMemcpy(D, Dh.data(), sizeof(double) * nn, hipMemcpyHostToDevice);
  expect(mderi_jkbuild(c, b, D, J, K, nao, E, nullptr, nullptr) == MDERI_OK, "jkbuild");
  const std::vector<double> Ja = host(J, nn), Ka = host(K, nn);
  expect(all_finite(Ja) && all_finite(Ka) && all_finite(host(E, 2)), "jkbuild finite");
  {
    mderi_opts o{};
    o.deterministic = 1;
    expect(mderi_jkbuild(c, b, D, J, K, nao, nullptr, &o, nullptr) == MDERI_OK, "jkbuild deterministic");
    expect(mderi_jkbuild(c, b, D, J2, K2, nao, nullptr, &o, nullptr) == MDERI_OK, "jkbuild deterministic again");
    const std::vector<double> j1 = host(J, nn), k1 = host(K, nn), j2 = host(J2, nn), k2 = host(K2, nn);
    expect(j1 == j2 && k1 == k2, "deterministic J and K repeat bitwise");
    expect(symmetric(j1, nao) && symmetric(k1, nao), "deterministic J and K symmetric");
    double d = 0.0, m = 0.0;
    for (size_t e = 0; e < nn; ++e) {
      d = std::fmax(d, std::fabs(k1[e] - Ka[e]));
      m = std::fmax(m, std::fabs(Ka[e]));
    }
    expect(d <= 1e-13 * m, "deterministic K agrees with the atomic K");
    o.deterministic = 3;
    expect(mderi_kbuild(c, b, D, K, nao, &o, nullptr) == MDERI_EINVAL, "deterministic 3 rejected");
  }
  expect(mderi_kbuild(c, b, D, K, nao, nullptr, nullptr) == MDERI_OK, "kbuild");
  expect(mderi_jkbuild(c, b, D, nullptr, nullptr, nao, nullptr, nullptr, nullptr) == MDERI_EINVAL,
         "jkbuild with no output");
  expect(mderi_kbuild(c, b, D, K, nao + 1, nullptr, nullptr) == MDERI_EINVAL, "kbuild wrong nao");
  double *G = dev(3 * (size_t)nsh);
  expect(mderi_kbuild_grad(c, b, MDERI_EXCHANGE, D, D, nao, 1.0, G, nsh, 0, nullptr, nullptr) == MDERI_OK,
         "kbuild_grad exchange");
  expect(mderi_kbuild_grad(c, b, MDERI_COULOMB, D, K, nao, 0.5, G, nsh, 1, nullptr, nullptr) == MDERI_OK,
         "kbuild_grad coulomb, unsymmetric weights, accumulate");
  expect(all_finite(host(G, 3 * (size_t)nsh)), "gradient finite");
  {
    mderi_opts o{};
    o.deterministic = 1;
    double *G2 = dev(3 * (size_t)nsh);
    expect(mderi_kbuild_grad(c, b, MDERI_EXCHANGE, D, D, nao, 1.0, G, nsh, 0, &o, nullptr) == MDERI_OK &&
               mderi_kbuild_grad(c, b, MDERI_EXCHANGE, D, D, nao, 1.0, G2, nsh, 0, &o, nullptr) == MDERI_OK,
           "kbuild_grad deterministic");
    expect(host(G, 3 * (size_t)nsh) == host(G2, 3 * (size_t)nsh), "deterministic gradient repeats bitwise");
    (void)hipFree(G2);
  }
  expect(mderi_kbuild_grad(c, b, 7, D, D, nao, 1.0, G, nsh, 0, nullptr, nullptr) == MDERI_EINVAL, "bad pattern");
  expect(mderi_dfj(c, b, a, D, J, nao, nullptr, nullptr) == MDERI_OK, "dfj");
  expect(all_finite(host(J, nn)) && symmetric(host(J, nn), nao), "dfj finite and symmetric");
  expect(mderi_dfk(c, b, a, D, K, nao, nullptr, nullptr) == MDERI_OK, "dfk");
  expect(all_finite(host(K, nn)) && symmetric(host(K, nn), nao), "dfk finite and symmetric");
  expect(mderi_dfk(c, b, a, D, K, nao + 1, nullptr, nullptr) == MDERI_EINVAL, "dfk wrong nao");

  // moved centres, timing, progress
  {
    std::vector<double> cen = s.centers;
    for (double &x : cen) x += 0.01;
    double *cd = dev(cen.size());
    (void)hipMemcpy(cd, cen.data(), sizeof(double) * cen.size(), hipMemcpyHostToDevice);
    expect(mderi_basis_set_centers(b, cd, nullptr) == MDERI_OK, "basis_set_centers");
    expect(mderi_kernel_timing(c, 1) == MDERI_OK, "kernel_timing on");
    expect(mderi_kbuild(c, b, D, K, nao, nullptr, nullptr) == MDERI_OK, "kbuild at moved centres");
    expect(mderi_kernel_timing(c, 0) == MDERI_OK, "kernel_timing off");
    int cnt = 0;
    expect(mderi_kernel_times(c, nullptr, 0, &cnt) == MDERI_OK, "kernel_times count");
    std::vector<double> ms(cnt > 0 ? cnt : 1);
    expect(mderi_kernel_times(c, ms.data(), (int)ms.size(), &cnt) == MDERI_OK, "kernel_times read");
    expect(mderi_progress(c, 0) == MDERI_OK, "progress off");
    (void)hipFree(cd);
  }

  // workspace cap: ENOMEM, then recovery
  expect(mderi_set_workspace_limit(c, 256) == MDERI_OK, "set_workspace_limit 256");
  expect(mderi_kbuild(c, b, D, K, nao, nullptr, nullptr) == MDERI_ENOMEM, "kbuild under the cap: ENOMEM");
  expect(mderi_eri4(c, b, 2, bra, 2, ket, V, nv, nullptr, nullptr) == MDERI_ENOMEM, "eri4 under the cap: ENOMEM");
  (void)hipDeviceSynchronize();
  expect(mderi_set_workspace_limit(c, 0) == MDERI_OK, "set_workspace_limit 0");
  expect(mderi_kbuild(c, b, D, K, nao, nullptr, nullptr) == MDERI_OK, "kbuild after the cap is lifted");

  (void)hipDeviceSynchronize();
  for (double *p : {V, Q, V3, B, V2, D, J, K, E, J2, K2, G}) (void)hipFree(p);
  mderi_basis_free(a);
  mderi_basis_free(b);
  mderi_destroy(c);
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}

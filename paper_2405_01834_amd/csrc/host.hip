// host.hip -- the C ABI of libmderi: contexts, basis upload, validation,
// class-batch planning and kernel dispatch.  Constant tables (Boys grid,
// Hermite order, Cartesian->solid coefficients) are generated here on the
// host from their mathematical definitions and uploaded once per context.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>
#include <map>
#include <array>
#include <numeric>
#include <memory>
#include <mutex>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "device_common.h"
#include "internal.h"

using namespace mderi;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static mderi_status fail(mderi_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(MDERI_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char *mderi_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// constant tables
// ---------------------------------------------------------------------------
namespace {

// Hermite functions (t,u,v) ordered by total degree, then t descending,
// then u descending.
std::vector<uint32_t> hermite_order() {
  std::vector<uint32_t> h;
  h.reserve(kNtilMax);
  for (int n = 0; n <= kLtotMax; ++n)
    for (int t = n; t >= 0; --t)
      for (int u = n - t; u >= 0; --u) h.push_back(pack3(t, u, n - t - u));
  return h;
}

// Real regular solid harmonics S_lm (S_00 = 1, same norm on the sphere as
// x^l) from the standard recurrences
//   S_{l+1,l+1}  = sqrt(2^{d(l,0)} (2l+1)/(2l+2)) (x S_{ll} - (1-d(l,0)) y S_{l,-l})
//   S_{l+1,-l-1} = sqrt(2^{d(l,0)} (2l+1)/(2l+2)) (y S_{ll} + (1-d(l,0)) x S_{l,-l})
//   S_{l+1,m}    = ((2l+1) z S_{lm} - sqrt((l+m)(l-m)) r^2 S_{l-1,m}) / sqrt((l+m+1)(l-m+1))
// Polynomials are dense coefficient arrays over monomials x^a y^b z^c of
// one degree, indexed by (a, b).
struct Poly {
  int deg = 0;
  std::vector<long double> c;  // [(deg+1)*(deg+1)], entry a*(deg+1)+b, c = deg-a-b
  explicit Poly(int d = 0) : deg(d), c((size_t)(d + 1) * (d + 1), 0.0L) {}
  long double &at(int a, int b) { return c[(size_t)a * (deg + 1) + b]; }
  long double get(int a, int b) const { return c[(size_t)a * (deg + 1) + b]; }
};
Poly mul_xyz(const Poly &p, int axis) {
  Poly r(p.deg + 1);
  for (int a = 0; a <= p.deg; ++a)
    for (int b = 0; a + b <= p.deg; ++b) {
      const long double v = p.get(a, b);
      if (v == 0.0L) continue;
      if (axis == 0) r.at(a + 1, b) += v;
      else if (axis == 1) r.at(a, b + 1) += v;
      else r.at(a, b) += v;
    }
  return r;
}
Poly mul_r2(const Poly &p) {
  Poly r(p.deg + 2);
  for (int a = 0; a <= p.deg; ++a)
    for (int b = 0; a + b <= p.deg; ++b) {
      const long double v = p.get(a, b);
      if (v == 0.0L) continue;
      r.at(a + 2, b) += v;
      r.at(a, b + 2) += v;
      r.at(a, b) += v;
    }
  return r;
}
Poly axpby(long double x, const Poly &p, long double y, const Poly &q) {
  Poly r(p.deg);
  for (size_t i = 0; i < r.c.size(); ++i) r.c[i] = x * p.c[i] + y * q.c[i];
  return r;
}

// S[l][m+l] for l <= lmax
std::vector<std::vector<Poly>> solid_harmonics(int lmax) {
  std::vector<std::vector<Poly>> S(lmax + 1);
  S[0].push_back(Poly(0));
  S[0][0].at(0, 0) = 1.0L;
  for (int l = 0; l < lmax; ++l) {
    std::vector<Poly> nx(2 * l + 3, Poly(l + 1));
    const long double f = sqrtl((l == 0 ? 2.0L : 1.0L) * (2 * l + 1) / (2.0L * l + 2.0L));
    const Poly &Sll = S[l][2 * l], &Slml = S[l][0];
    if (l == 0) {
      nx[2 * l + 2] = axpby(f, mul_xyz(Sll, 0), 0.0L, mul_xyz(Sll, 0));
      nx[0] = axpby(f, mul_xyz(Sll, 1), 0.0L, mul_xyz(Sll, 1));
    } else {
      nx[2 * l + 2] = axpby(f, mul_xyz(Sll, 0), -f, mul_xyz(Slml, 1));
      nx[0] = axpby(f, mul_xyz(Sll, 1), f, mul_xyz(Slml, 0));
    }
    for (int m = -l; m <= l; ++m) {
      Poly zs = mul_xyz(S[l][m + l], 2);
      Poly t(l + 1);
      if (l >= 1 && m >= -(l - 1) && m <= l - 1) t = mul_r2(S[l - 1][m + l - 1]);
      const long double den = sqrtl((long double)(l + m + 1) * (l - m + 1));
      const long double s = sqrtl((long double)(l + m) * (l - m));
      nx[m + l + 1] = axpby((2 * l + 1) / den, zs, -s / den, t);
    }
    S[l + 1] = nx;
  }
  return S;
}

// Boys table F_m(T_i) in long double: positive-term series for the largest
// m, F_m(T) = e^{-T} sum_k (2T)^k / [(2m+1)(2m+3)...(2m+2k+1)], then the
// downward recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).
std::vector<double> boys_table() {
  std::vector<double> tab((size_t)(kBoysNgrid + 1) * kBoysM);
  // last row: (2m-1)!! for F_m(T) = (2m-1)!! / (2T)^m F_0(T), T >= kBoysTmax
  {
    long double df = 1.0L;
    for (int m = 0; m < kBoysM; ++m) {
      tab[(size_t)kBoysNgrid * kBoysM + m] = (double)df;
      df *= 2 * m + 1;
    }
  }
  const int M = kBoysM - 1;
  for (int i = 0; i < kBoysNgrid; ++i) {
    const long double T = (long double)i / kBoysGridPerUnit;
    const long double et = expl(-T);
    long double term = 1.0L / (2 * M + 1), sum = term;
    for (int k = 1; k < 10000; ++k) {
      term *= 2.0L * T / (2 * M + 2 * k + 1);
      sum += term;
      if (k > T && term < 1e-24L * sum) break;
    }
    long double f = et * sum;
    tab[(size_t)i * kBoysM + M] = (double)f;
    for (int m = M - 1; m >= 0; --m) {
      f = (2.0L * T * f + et) / (2 * m + 1);
      tab[(size_t)i * kBoysM + m] = (double)f;
    }
  }
  return tab;
}

double dfact_odd(int n) {
  double r = 1.0;
  for (int i = n; i > 1; i -= 2) r *= i;
  return r;
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  hipError_t e = hipMalloc((void **)dst, sizeof(T) * (src.empty() ? 1 : src.size()));
  if (e != hipSuccess) return e;
  if (src.empty()) return hipSuccess;
  return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
enum WsSlot {
  WS_META, WS_G_BRA, WS_G_KET, WS_H_BRA, WS_H_KET, WS_DIAG, WS_KTMP, WS_QALL, WS_PAIRS, WS_HS, WS_HEXP, WS_HROW,
  WS_GPART, WS_DFB, WS_DFM, WS_DFT, WS_DFV, WS_DFI, WS_DFK1, WS_DFK2, WS_DFK3,
  WS_COUNT
};

struct TaskPlan;
void free_plan(TaskPlan *p);

// Scratch of the allocation-free entry point mderi_eri4_noalloc: every
// device region of that call (pair lists, primitive-pair data G and the
// transform matrices H of both sides) is a slice of this file-scope array.
// Each GPU holds its own copy from the first use of the library until the
// process ends.  Host code never passes `scratch` itself to a kernel (its
// name is a host-side stand-in there): mderi_create looks up this device's
// address once with hipGetSymbolAddress and keeps it in the context.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
// Pinned host staging allocated when a context is created, so that the
// allocation-free entry point can upload its metadata without allocating.
constexpr size_t kStageInitBytes = (size_t)4 << 20;  // per slot
constexpr int kStageSlots = 4;
constexpr size_t kPairCacheKeys = 2;  // pair selections a context keeps

namespace {
struct PairSets;  // a Schwarz pair selection (defined with select_pairs)
}  // namespace

struct mderi_ctx {
  int device = 0;
  Tables tab;
  void *ws[WS_COUNT] = {};
  size_t ws_cap[WS_COUNT] = {};
  size_t ws_limit = 0;  // cap on the sum of ws_cap (0 = none)
  // pinned staging for per-call host->device uploads: kStageSlots slots of
  // stage_cap bytes used in turn, each guarded by an event, so the host can
  // prepare the next calls while earlier uploads are still queued
  char *stage = nullptr;     // kStageSlots * stage_cap bytes
  size_t stage_cap = 0;      // bytes per slot (the most one call can stage)
  hipEvent_t stage_done[kStageSlots] = {};
  bool stage_pending[kStageSlots] = {};
  int stage_slot = 0;        // slot of the current call
  char *stage_cur = nullptr;  // its base
  // kernel timing: when on, each fused-kernel launch is bracketed by a pair
  // of events on its stream (pairs are recycled after they are read)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free;
  bool progress = false;  // report finished launch groups of the quartet engine
  // task-list plans of mderi_eri3_batch, most recent last, and the tile
  // choices of the autotuner per class signature
  std::vector<TaskPlan *> plans;
  std::map<std::array<int, 6>, std::array<int, 3>> tune;
  hipStream_t cap_stream = nullptr;  // stream used to capture graphs
  std::vector<hipStream_t> side;     // side streams of concurrent task-list groups
  uint64_t next_serial = 1;
  char *scratch = nullptr;  // device address of `scratch` on this context's device
  rocblas_handle blas = nullptr;  // library handle of the density-fitting solve (created on first use)
  // Schwarz pair selections of the last kPairCacheKeys (basis upload,
  // geometry, tau) keys, most recent last: a J/K or gradient call on a basis
  // whose centres have not moved since reuses its selection without the
  // device-to-host copy and the wait it needs.  Upload serials are never
  // reused, so an entry of a freed basis matches nothing; it stays (host
  // memory only) until newer keys push it out or the context is destroyed.
  struct PairCacheEntry {
    uint64_t serial, geom;
    double tau;
    std::shared_ptr<const PairSets> ps;
  };
  std::vector<PairCacheEntry> pair_cache;
  // density-fitting factors of the last (basis, fitting basis) pair, kept in
  // the DF work space slots for the next mderi_dfj / mderi_dfk call on the
  // same pair and geometries: df_stage 0 = none, 1 = the (ab|P) matrix B and
  // the Cholesky factor L of the metric, 2 = B' = B L^-T in place of B,
  // 3 = B' also spread over all AO pairs for the exchange contractions
  uint64_t df_key[4] = {};  // basis serial and geometry, fitting basis serial and geometry
  int df_stage = 0, df_nrow = 0;
};

struct mderi_basis {
  mderi_ctx *ctx = nullptr;
  uint64_t serial = 0;  // unique per upload (keys cached task plans)
  uint64_t geom = 0;    // bumped whenever the centres change (keys cached pair selections)
  int nshell = 0, nao = 0;
  std::vector<int> l, K, poff, atom, ao_off;
  DevBasis dev;
};

static mderi_status ws_get(mderi_ctx *c, int slot, size_t bytes, void **out) {
  if (bytes == 0) bytes = 16;
  if (c->ws_cap[slot] < bytes) {
    if (c->ws_limit) {
      size_t others = 0;
      for (int i = 0; i < WS_COUNT; ++i)
        if (i != slot) others += c->ws_cap[i];
      if (others + bytes > c->ws_limit)
        return fail(MDERI_ENOMEM, "device workspace of %zu bytes would exceed the limit of %zu bytes (%zu held)",
                    bytes, c->ws_limit, others);
    }
    if (c->ws[slot]) {
      HIP_TRY(hipDeviceSynchronize());
      HIP_TRY(hipFree(c->ws[slot]));
      c->ws[slot] = nullptr;
      c->ws_cap[slot] = 0;
    }
    size_t cap = bytes + bytes / 4;
    if (c->ws_limit) {
      size_t others = 0;
      for (int i = 0; i < WS_COUNT; ++i)
        if (i != slot) others += c->ws_cap[i];
      cap = std::min(cap, c->ws_limit - others);
    }
    if (hipMalloc(&c->ws[slot], cap) != hipSuccess) {
      (void)hipGetLastError();
      return fail(MDERI_ENOMEM, "device workspace of %zu bytes could not be allocated", cap);
    }
    c->ws_cap[slot] = cap;
  }
  *out = c->ws[slot];
  return MDERI_OK;
}

// Copies `n` host bytes to device `dst` on `s` through the current staging
// slot (stage_begin .. stage_end).
static mderi_status stage_copy(mderi_ctx *c, void *dst, const void *src, size_t n, hipStream_t s, size_t *used) {
  if (*used + n > c->stage_cap) return fail(MDERI_EINVAL, "internal: staging overflow");
  memcpy(c->stage_cur + *used, src, n);
  HIP_TRY(hipMemcpyAsync(dst, c->stage_cur + *used, n, hipMemcpyHostToDevice, s));
  *used += (n + 255) & ~(size_t)255;
  return MDERI_OK;
}

// Takes the next staging slot for a call that stages `need` bytes: waits for
// the uploads that last used the slot (kStageSlots calls back), or for all of
// them when the slots must grow.
static mderi_status stage_begin(mderi_ctx *c, size_t need) {
  if (need > c->stage_cap) {
    for (int k = 0; k < kStageSlots; ++k)
      if (c->stage_pending[k]) {
        HIP_TRY(hipEventSynchronize(c->stage_done[k]));
        c->stage_pending[k] = false;
      }
    if (c->stage) HIP_TRY(hipHostFree(c->stage));
    c->stage = nullptr;
    c->stage_cap = 0;
    const size_t cap = (need + need / 2 + 4096 + 255) & ~(size_t)255;
    HIP_TRY(hipHostMalloc((void **)&c->stage, cap * kStageSlots, hipHostMallocDefault));
    c->stage_cap = cap;
  }
  const int k = c->stage_slot;
  if (c->stage_pending[k]) {
    HIP_TRY(hipEventSynchronize(c->stage_done[k]));
    c->stage_pending[k] = false;
  }
  c->stage_cur = c->stage + (size_t)k * c->stage_cap;
  return MDERI_OK;
}

static mderi_status stage_end(mderi_ctx *c, hipStream_t s) {
  const int k = c->stage_slot;
  HIP_TRY(hipEventRecord(c->stage_done[k], s));
  c->stage_pending[k] = true;
  c->stage_slot = (k + 1) % kStageSlots;
  return MDERI_OK;
}

extern "C" mderi_status mderi_create(int device, mderi_ctx_t *out) {
  if (!out) return fail(MDERI_EINVAL, "mderi_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(MDERI_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(MDERI_EINVAL, "device %d out of range [0,%d)", device, ndev);
  HIP_TRY(hipSetDevice(device));
  mderi_ctx *c = new mderi_ctx;
  c->device = device;

  std::vector<uint32_t> herm = hermite_order();
  std::vector<double> boys = boys_table();
  auto S = solid_harmonics(kLshell);
  // nonzeros of slot s = l*(2*kLshell+1) + (m+l) occupy [sstart[s], sstart[s+1])
  std::vector<int> sstart(kSolidSlots, 0);
  std::vector<double> scoef;
  std::vector<uint32_t> scart;
  for (int sl = 0; sl < kSolidSlots - 1; ++sl) {
    sstart[sl] = (int)scoef.size();
    const int l = sl / (2 * kLshell + 1), mm = sl % (2 * kLshell + 1);
    if (mm > 2 * l) continue;
    long double mx = 0.0L;
    for (auto &pl : S[l])
      for (long double v : pl.c) mx = fmaxl(mx, fabsl(v));
    const Poly &p = S[l][mm];
    for (int a = l; a >= 0; --a)
      for (int bb = l - a; bb >= 0; --bb) {
        const long double v = p.get(a, bb);
        if (fabsl(v) > 1e-13L * mx) {
          scoef.push_back((double)v);
          scart.push_back(pack3(a, bb, l - a - bb));
        }
      }
  }
  sstart[kSolidSlots - 1] = (int)scoef.size();
  hipError_t e;
  if ((e = upload(&c->tab.herm, herm)) != hipSuccess || (e = upload(&c->tab.boys, boys)) != hipSuccess ||
      (e = upload(&c->tab.solid_start, sstart)) != hipSuccess || (e = upload(&c->tab.solid_coef, scoef)) != hipSuccess ||
      (e = upload(&c->tab.solid_cart, scart)) != hipSuccess) {
    mderi_destroy(c);
    return fail(MDERI_EDEVICE, "table upload failed: %s", hipGetErrorString(e));
  }
  for (int k = 0; k < kStageSlots; ++k)
    if ((e = hipEventCreateWithFlags(&c->stage_done[k], hipEventDisableTiming)) != hipSuccess) {
      mderi_destroy(c);
      return fail(MDERI_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  // this device's copy of the scratch array (the device is current here)
  if ((e = hipGetSymbolAddress((void **)&c->scratch, HIP_SYMBOL(scratch))) != hipSuccess || !c->scratch) {
    mderi_destroy(c);
    return fail(MDERI_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }
  if ((e = hipHostMalloc((void **)&c->stage, kStageInitBytes * kStageSlots, hipHostMallocDefault)) != hipSuccess) {
    c->stage = nullptr;
    mderi_destroy(c);
    return fail(MDERI_ENOMEM, "pinned staging of %zu bytes: %s", kStageInitBytes * kStageSlots,
                hipGetErrorString(e));
  }
  c->stage_cap = kStageInitBytes;
  *out = c;
  g_err.clear();
  return MDERI_OK;
}

extern "C" void mderi_destroy(mderi_ctx_t c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(c->tab.boys);
  (void)hipFree(c->tab.herm);
  (void)hipFree(c->tab.solid_start);
  (void)hipFree(c->tab.solid_coef);
  (void)hipFree(c->tab.solid_cart);
  for (int i = 0; i < WS_COUNT; ++i) (void)hipFree(c->ws[i]);
  if (c->stage) (void)hipHostFree(c->stage);
  for (hipEvent_t e : c->stage_done)
    if (e) (void)hipEventDestroy(e);
  for (TaskPlan *p : c->plans) free_plan(p);
  if (c->blas) (void)rocblas_destroy_handle(c->blas);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipStream_t x : c->side) (void)hipStreamDestroy(x);
  for (auto *v : {&c->ev_used, &c->ev_free})
    for (auto &e : *v) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  delete c;
}

extern "C" mderi_status mderi_kernel_timing(mderi_ctx_t c, int enable) {
  if (!c) return fail(MDERI_EINVAL, "mderi_kernel_timing: NULL context");
  c->timing = enable != 0;
  return MDERI_OK;
}

// Autotune cache file: a header line "mderi-tune <format> <device arch>", the
// entry count, then one line per class signature: the six key integers
// (l_a l_b l_c l_d, -1 for a 1-centre side, and the largest primitive-pair
// counts of the two sides) and the three tile integers (npt nps dbuf).
static constexpr int kTuneFormat = 1;

static std::string device_arch(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  for (char &ch : a)
    if (ch == ' ') ch = '_';
  return a;
}

extern "C" mderi_status mderi_tune_save(mderi_ctx_t c, const char *path) {
  if (!c || !path) return fail(MDERI_EINVAL, "mderi_tune_save: NULL context or path");
  FILE *f = std::fopen(path, "w");
  if (!f) return fail(MDERI_EINVAL, "mderi_tune_save: cannot open %s for writing", path);
  bool ok = std::fprintf(f, "mderi-tune %d %s\n%zu\n", kTuneFormat, device_arch(c->device).c_str(), c->tune.size()) > 0;
  for (const auto &kv : c->tune) {
    const auto &k = kv.first;
    const auto &v = kv.second;
    ok = ok && std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", k[0], k[1], k[2], k[3], k[4], k[5], v[0], v[1], v[2]) > 0;
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(MDERI_EINVAL, "mderi_tune_save: writing %s failed", path);
  return MDERI_OK;
}

extern "C" mderi_status mderi_tune_load(mderi_ctx_t c, const char *path) {
  if (!c || !path) return fail(MDERI_EINVAL, "mderi_tune_load: NULL context or path");
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(MDERI_EINVAL, "mderi_tune_load: cannot open %s", path);
  char arch[256] = {0};
  int format = 0;
  long n = -1;
  if (std::fscanf(f, "mderi-tune %d %255s %ld", &format, arch, &n) != 3 || format != kTuneFormat || n < 0 ||
      n > 1000000) {
    std::fclose(f);
    return fail(MDERI_EINVAL, "mderi_tune_load: %s is not an autotune cache of format %d", path, kTuneFormat);
  }
  if (device_arch(c->device) != arch) {
    std::fclose(f);
    return fail(MDERI_EINVAL, "mderi_tune_load: %s was written on %s, this device is %s", path, arch,
                device_arch(c->device).c_str());
  }
  std::vector<std::pair<std::array<int, 6>, std::array<int, 3>>> got;
  for (long e = 0; e < n; ++e) {
    std::array<int, 6> k;
    std::array<int, 3> v;
    if (std::fscanf(f, "%d %d %d %d %d %d %d %d %d", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &v[0], &v[1],
                    &v[2]) != 9) {
      std::fclose(f);
      return fail(MDERI_EINVAL, "mderi_tune_load: %s: entry %ld of %ld is malformed", path, e, n);
    }
    got.push_back({k, v});
  }
  std::fclose(f);
  // a choice is only ever used when it is among the class's candidates, so a
  // stale entry costs nothing; nothing is changed unless the whole file parsed
  for (const auto &kv : got) c->tune[kv.first] = kv.second;
  return MDERI_OK;
}

extern "C" mderi_status mderi_set_workspace_limit(mderi_ctx_t c, size_t bytes) {
  if (!c) return fail(MDERI_EINVAL, "mderi_set_workspace_limit: NULL context");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipDeviceSynchronize());
  c->df_stage = 0;  // the kept density-fitting factors go with the work space
  for (int i = 0; i < WS_COUNT; ++i) {
    if (c->ws[i]) HIP_TRY(hipFree(c->ws[i]));
    c->ws[i] = nullptr;
    c->ws_cap[i] = 0;
  }
  c->ws_limit = bytes;
  return MDERI_OK;
}

extern "C" mderi_status mderi_progress(mderi_ctx_t c, int enable) {
  if (!c) return fail(MDERI_EINVAL, "mderi_progress: NULL context");
  c->progress = enable != 0;
  return MDERI_OK;
}

extern "C" mderi_status mderi_kernel_times(mderi_ctx_t c, double *ms_host, int cap, int *count) {
  if (!c || !count) return fail(MDERI_EINVAL, "mderi_kernel_times: NULL context or count");
  if (cap > 0 && !ms_host) return fail(MDERI_EINVAL, "mderi_kernel_times: NULL output with cap %d", cap);
  HIP_TRY(hipSetDevice(c->device));
  const int n = (int)c->ev_used.size();
  *count = n;
  for (int i = 0; i < n; ++i) {
    auto &e = c->ev_used[i];
    if (i < cap) {
      HIP_TRY(hipEventSynchronize(e.second));
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
      ms_host[i] = ms;
    }
  }
  if (cap >= n) {
    c->ev_free.insert(c->ev_free.end(), c->ev_used.begin(), c->ev_used.end());
    c->ev_used.clear();
  }
  return MDERI_OK;
}

// ---------------------------------------------------------------------------
// basis
// ---------------------------------------------------------------------------
extern "C" mderi_status mderi_basis_upload(mderi_ctx_t c, int nshell, const int *l, const int *nprim,
                                           const double *exps, const double *coefs, const double *centers,
                                           const int *atom, int normalize, mderi_basis_t *out) {
  if (!c || !out) return fail(MDERI_EINVAL, "mderi_basis_upload: NULL context or out");
  *out = nullptr;
  if (nshell <= 0) return fail(MDERI_EINVAL, "nshell must be positive (got %d)", nshell);
  if (!l || !nprim || !exps || !coefs || !centers) return fail(MDERI_EINVAL, "mderi_basis_upload: NULL array");
  mderi_basis *b = new mderi_basis;
  b->ctx = c;
  b->serial = c->next_serial++;
  b->nshell = nshell;
  b->l.assign(l, l + nshell);
  b->K.assign(nprim, nprim + nshell);
  b->poff.resize(nshell);
  b->atom.resize(nshell);
  b->ao_off.resize(nshell);
  int np = 0;
  for (int i = 0; i < nshell; ++i) {
    if (l[i] < 0 || l[i] > kLmax) {
      delete b;
      return fail(MDERI_EUNSUPPORTED, "shell %d: l=%d outside [0,%d]", i, l[i], kLmax);
    }
    if (nprim[i] < 1 || nprim[i] > MDERI_KMAX) {
      delete b;
      return fail(MDERI_EUNSUPPORTED, "shell %d: %d primitives outside [1,%d]", i, nprim[i], MDERI_KMAX);
    }
    b->poff[i] = np;
    np += nprim[i];
    b->ao_off[i] = b->nao;
    b->nao += 2 * l[i] + 1;
    b->atom[i] = atom ? atom[i] : i;
    for (int x = 0; x < 3; ++x)
      if (!std::isfinite(centers[3 * i + x])) {
        delete b;
        return fail(MDERI_EINVAL, "shell %d: non-finite centre", i);
      }
  }
  std::vector<double> cn(np), ex(exps, exps + np);
  for (int i = 0; i < nshell; ++i) {
    const int L = l[i], K = nprim[i], o = b->poff[i];
    for (int k = 0; k < K; ++k)
      if (!(std::isfinite(exps[o + k]) && exps[o + k] > 0.0) || !std::isfinite(coefs[o + k])) {
        delete b;
        return fail(MDERI_EINVAL, "shell %d primitive %d: exponent must be finite and > 0, coefficient finite", i, k);
      }
    if (!normalize) {
      for (int k = 0; k < K; ++k) cn[o + k] = coefs[o + k];
      continue;
    }
    // unit-normalised primitives x^l e^{-z r^2}: (2z/pi)^{3/4} (4z)^{l/2} / sqrt((2l-1)!!),
    // then the contraction rescaled to unit norm; two such primitives on one
    // centre overlap by (2 sqrt(z z') / (z + z'))^{l + 3/2}.
    double norm2 = 0.0;
    for (int k = 0; k < K; ++k)
      for (int kk = 0; kk < K; ++kk) {
        const double zk = exps[o + k], zkk = exps[o + kk];
        norm2 += coefs[o + k] * coefs[o + kk] * std::pow(2.0 * std::sqrt(zk * zkk) / (zk + zkk), L + 1.5);
      }
    if (!(norm2 > 0.0)) {
      delete b;
      return fail(MDERI_EINVAL, "shell %d: contraction has zero norm", i);
    }
    const double inv = 1.0 / std::sqrt(norm2);
    for (int k = 0; k < K; ++k) {
      const double z = exps[o + k];
      cn[o + k] = inv * coefs[o + k] * std::pow(2.0 * z / M_PI, 0.75) * std::pow(4.0 * z, 0.5 * L) /
                  std::sqrt(dfact_odd(2 * L - 1));
    }
  }
  hipError_t e = hipSetDevice(c->device);
  std::vector<double> cen(centers, centers + 3 * nshell);
  b->dev.nshell = nshell;
  b->dev.nprim = np;
  if (e == hipSuccess) e = upload(&b->dev.l, b->l);
  if (e == hipSuccess) e = upload(&b->dev.K, b->K);
  if (e == hipSuccess) e = upload(&b->dev.poff, b->poff);
  if (e == hipSuccess) e = upload(&b->dev.atom, b->atom);
  if (e == hipSuccess) e = upload(&b->dev.ao_off, b->ao_off);
  if (e == hipSuccess) e = upload(&b->dev.centers, cen);
  if (e == hipSuccess) e = upload(&b->dev.exps, ex);
  if (e == hipSuccess) e = upload(&b->dev.coefs, cn);
  if (e != hipSuccess) {
    mderi_basis_free(b);
    return fail(MDERI_EDEVICE, "basis upload: %s", hipGetErrorString(e));
  }
  *out = b;
  return MDERI_OK;
}

extern "C" void mderi_basis_free(mderi_basis_t b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(b->dev.l);
  (void)hipFree(b->dev.K);
  (void)hipFree(b->dev.poff);
  (void)hipFree(b->dev.atom);
  (void)hipFree(b->dev.ao_off);
  (void)hipFree(b->dev.centers);
  (void)hipFree(b->dev.exps);
  (void)hipFree(b->dev.coefs);
  delete b;
}

extern "C" int mderi_basis_nshell(mderi_basis_t b) { return b ? b->nshell : 0; }
extern "C" int mderi_basis_nao(mderi_basis_t b) { return b ? b->nao : 0; }

// ---------------------------------------------------------------------------
// class batches
// ---------------------------------------------------------------------------
namespace {

// Validates a pair list of one class and expands it into primitive pairs.
mderi_status expand_pairs(const mderi_basis *b, int n, const int32_t *pairs, const char *what, int *la, int *lb,
                          std::vector<PrimPair> &pp, std::vector<int> &off) {
  if (n <= 0) return fail(MDERI_EINVAL, "%s: need at least one pair (got %d)", what, n);
  if (!pairs) return fail(MDERI_EINVAL, "%s: NULL pair list", what);
  pp.clear();
  off.assign(1, 0);
  for (int i = 0; i < n; ++i) {
    const int s0 = pairs[2 * i], s1 = pairs[2 * i + 1];
    if (s0 < 0 || s0 >= b->nshell || s1 < 0 || s1 >= b->nshell)
      return fail(MDERI_EINVAL, "%s: pair %d = (%d,%d) out of range [0,%d)", what, i, s0, s1, b->nshell);
    if (i == 0) {
      *la = b->l[s0];
      *lb = b->l[s1];
    } else if (b->l[s0] != *la || b->l[s1] != *lb) {
      return fail(MDERI_EINVAL, "%s: pair %d has class (%d,%d) but the batch is (%d,%d)", what, i, b->l[s0],
                  b->l[s1], *la, *lb);
    }
    for (int ka = 0; ka < b->K[s0]; ++ka)
      for (int kb = 0; kb < b->K[s1]; ++kb) pp.push_back(PrimPair{s0, s1, b->poff[s0] + ka, b->poff[s1] + kb});
    off.push_back((int)pp.size());
  }
  return MDERI_OK;
}

}  // namespace

namespace {

// Whether t*s1 + u*s2 + v is injective on |r| = t+u+v <= L.
bool cube_injective(int L, int s1, int s2, std::vector<char> &seen) {
  seen.assign((size_t)L * s1 + (size_t)L * s2 + L + 1, 0);
  for (int t = 0; t <= L; ++t)
    for (int u = 0; u <= L - t; ++u)
      for (int v = 0; v <= L - t - u; ++v) {
        char &x = seen[(size_t)t * s1 + (size_t)u * s2 + v];
        if (x) return false;
        x = 1;
      }
  return true;
}

// [r] cube strides for total angular momentum L: any (S1, S2) that keeps
// t*S1 + u*S2 + v injective on |r| <= L makes the offset additive, so [p+q]
// is found at offset(p) + offset(q) (S2 > L, S1 > L*S2 always works; smaller
// S1 that stay injective give a cube up to a quarter smaller).  Among
// injective strides near the smallest, pick the pair whose bra offsets
// (|p| <= Lb) fall most evenly into the 16 LDS bank pairs that one 16-lane
// group of a 64-bit read spans, then the smallest cube.  Cached per (L, Lb).
void choose_cube(int L, int Lb, int *S1, int *S2) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::pair<int, int>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({L, Lb});
  if (it != cache.end()) {
    *S1 = it->second.first;
    *S2 = it->second.second;
    return;
  }
  const int n = ntil(Lb), nt = (n + 15) / 16;
  long best_key = -1;
  std::vector<char> seen;
  for (int s2 = L + 1; s2 <= L + 16; ++s2) {
    int s1min = s2 + 1;
    while (s1min <= L * s2 + 1 && !cube_injective(L, s1min, s2, seen)) ++s1min;
    for (int s1 = s1min; s1 <= s1min + 24; ++s1) {
      if (s1 > s1min && !cube_injective(L, s1, s2, seen)) continue;
      int hist[16] = {0};
      for (int d = 0; d <= Lb; ++d)
        for (int t = d; t >= 0; --t)
          for (int u = d - t; u >= 0; --u) ++hist[(t * s1 + u * s2 + (d - t - u)) % 16];
      int mx = 0;
      for (int r = 0; r < 16; ++r) mx = hist[r] > mx ? hist[r] : mx;
      const long excess = mx > nt ? mx - nt : 0;
      const long key = excess * 100000000L + (long)L * s1;
      if (best_key < 0 || key < best_key) {
        best_key = key;
        *S1 = s1;
        *S2 = s2;
      }
    }
  }
  cache[{L, Lb}] = {*S1, *S2};
}

// Row order of the bra Hermite functions for tiles of 16 rows: functions
// sorted by bank (offset mod 16) are dealt round-robin over the tiles, so a
// tile holds at most ceil(bucket/ntiles) functions of one bank; padding rows
// (kPadRow) reuse functions of banks the tile does not use yet.
std::vector<uint32_t> bra_row_order(int Lb, int S1, int S2, int Nh_pad) {
  std::vector<uint32_t> p;
  for (int d = 0; d <= Lb; ++d)
    for (int t = d; t >= 0; --t)
      for (int u = d - t; u >= 0; --u) p.push_back(pack3(t, u, d - t - u));
  auto bank = [&](uint32_t h) { return (int)(((h & 0xff) * S1 + ((h >> 8) & 0xff) * S2 + ((h >> 16) & 0xff)) % 16); };
  std::vector<int> idx(p.size());
  for (size_t i = 0; i < p.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return bank(p[x]) < bank(p[y]); });
  const int nt = Nh_pad / 16;
  std::vector<std::vector<uint32_t>> tiles(nt);
  for (size_t k = 0; k < idx.size(); ++k) tiles[k % nt].push_back(p[idx[k]]);
  std::vector<int> by_bank[16];
  for (uint32_t h : p) by_bank[bank(h)].push_back(h);
  std::vector<uint32_t> out;
  out.reserve(Nh_pad);
  for (auto &tl : tiles) {
    bool used[16] = {false};
    for (uint32_t h : tl) used[bank(h)] = true;
    int r = 0;
    while (tl.size() < 16) {
      while (r < 16 && (used[r] || by_bank[r].empty())) ++r;
      if (r < 16) {
        tl.push_back(by_bank[r][0] | kPadRow);
        used[r] = true;
      } else {
        tl.push_back(p[0] | kPadRow);
      }
    }
    out.insert(out.end(), tl.begin(), tl.end());
  }
  return out;
}

// One side of a class batch: shell pairs of one class (or single shells of
// one l when one_centre) expanded into primitive pairs.
struct Side {
  const mderi_basis *b;
  int la, lb;
  bool one_centre;
  std::vector<PrimPair> pp;
  std::vector<int> off;
};

// Top-degree Hermite functions of degree l (t, then u descending), the only
// ones a single solid-harmonic Gaussian expands into (Hobson's theorem; the
// lower rows of its transform matrix vanish identically), padded with
// kPadRow to a multiple of 8.
std::vector<uint32_t> top_degree_rows(int l) {
  std::vector<uint32_t> r;
  for (int t = l; t >= 0; --t)
    for (int u = l - t; u >= 0; --u) r.push_back(pack3(t, u, l - t - u));
  while (r.size() % 8) r.push_back(kPadRow);
  return r;
}

// Enqueues pair data (bra and ket) and the fused kernel for one class batch.
// diag != 0 evaluates only (ij|ij) (bra list == ket list) and writes the
// diagonal [ij][ab] to V.

// Launches the fused kernel, bracketed by timing events when timing is on.
mderi_status launch_eri4_timed(mderi_ctx *c, const Eri4Args &ea, hipStream_t s) {
  if (c->timing) {
    if (c->ev_free.empty()) {
      std::pair<hipEvent_t, hipEvent_t> e;
      HIP_TRY(hipEventCreate(&e.first));
      HIP_TRY(hipEventCreate(&e.second));
      c->ev_free.push_back(e);
    }
    const auto e = c->ev_free.back();
    c->ev_free.pop_back();
    c->ev_used.push_back(e);
    HIP_TRY(hipEventRecord(e.first, s));
    HIP_TRY(launch_eri4(ea, s));
    HIP_TRY(hipEventRecord(e.second, s));
  } else {
    HIP_TRY(launch_eri4(ea, s));
  }
  return MDERI_OK;
}

std::vector<std::array<int, 3>> block_candidates(int Nhb, int Nb, int Nk, int L, int cube_sz, int Nhk_pad,
                                                 int maxpp);

// noalloc: every device region is a slice of the context's scratch array and
// the metadata goes through the staging buffer as it is (the allocation-free
// entry point); otherwise regions come from the pooled workspace.
// tile_variant > 0 forces that work split (see mderi_eri4_tile_variants);
// count_only stores the number of splits in *count and enqueues nothing.
#ifndef MDERI_QUARTET_RUN
#define MDERI_QUARTET_RUN 4
#endif
// Quartet runs and V stored from registers (Eri4Args::nrun, vdirect) for one
// work split of a class batch whose pairs have at most maxb / maxk primitive
// pairs (maxpp their sum): both need single-primitive bra pairs and plain
// class-batch output, runs also single-primitive kets and two [r] cubes, V
// from registers one row part.  Column-slab classes are left out: their
// [r] cube is too large for two copies (L >= 20), so runs would not overlap.  Off again if the run's ket data would push
// the workgroup past the LDS limit.  Measured on the 65,536-quartet K=1
// batches, runs of 4 against none: [dd|dd] 1.32x, [ff|ff] 1.24x, [gg|gg]
// 1.12x (runs of 8 within 2% of 4).
void set_run_mode(Eri4Args &a, int maxb, int maxk, int maxpp) {
  const bool single = maxb == 1 && !a.diag && a.nslab == 1 && !a.bra_Hs && !a.orow;
  // (buffer stores of V: one quartet's nbra Nb Nk doubles within 2 GiB)
  a.vdirect = single && a.nps == 1 && (long)a.nbra * a.Nb * a.Nk * 8 < (1L << 31) ? 1 : 0;
  // runs shorten the grid: keep at least 2048 workgroups (8 per CU)
  const long nrun = std::min<long>(MDERI_QUARTET_RUN, (long)a.nbra * a.nket / 2048);
  a.nrun = single && maxk == 1 && a.dbuf && nrun > 1 ? (int)nrun : 0;
  a.maxpp = std::max(maxpp, a.nrun > 1 ? 1 + a.nrun : 0);
  if (eri4_lds_bytes(a) > 160 * 1024) {
    a.nrun = 0;
    a.maxpp = maxpp;
  }
}

mderi_status run_class_batch(mderi_ctx *c, const Side &bra, const Side &ket, int diag, double *V,
                             const std::vector<int> *extra_idx, void **d_extra_idx, hipStream_t s, int flags = 0,
                             int precision = 0, int slices = kSplitDefault, bool noalloc = false, int tile_variant = 0,
                             int *count = nullptr) {
  const int nbra = (int)bra.off.size() - 1, nket = (int)ket.off.size() - 1;
  const int la = bra.la, lb = bra.one_centre ? 0 : bra.lb, lc = ket.la, ld = ket.one_centre ? 0 : ket.lb;
  const int Lb = la + lb, Lk = lc + ld, L = Lb + Lk;
  const int Nb = nsph(la) * nsph(lb), Nk = ket.one_centre ? nsph(lc) : nsph(lc) * nsph(ld);
  const int Nhb = ntil(Lb);
  const std::vector<uint32_t> korder = ket.one_centre ? top_degree_rows(lc) : std::vector<uint32_t>();
  const int Nhk = ket.one_centre ? (lc + 1) * (lc + 2) / 2 : ntil(Lk);
  const int Nhk_pad = (Nhk + 7) & ~7;
  int S1 = 1, S2 = 1;
  choose_cube(L, Lb, &S1, &S2);
  const int cube_sz = (L * S1 + 2) & ~1;
  int maxb = 0, maxk = 0;
  for (int i = 0; i < nbra; ++i) maxb = std::max(maxb, bra.off[i + 1] - bra.off[i]);
  for (int i = 0; i < nket; ++i) maxk = std::max(maxk, ket.off[i + 1] - ket.off[i]);
  const int maxpp = maxb + maxk;
  Eri4Plan pl{};
  if (!eri4_plan(Nhb, Nb, Nk, L, cube_sz, Nhk_pad, maxpp, true, &pl))
    return fail(MDERI_EUNSUPPORTED, "class (%d%d|%d%d) is beyond the fused kernel's tiles", la, lb, lc, ld);
  // tile variants: the tuned choice for this class signature, or all of
  // them timed on this batch when autotuning (single-slab classes only)
  const bool split = precision == MDERI_SPLIT_BF16;
  if (split && (pl.npt & 1)) ++pl.npt;  // the BF16 operands pair 16-row tiles
  std::vector<std::array<int, 3>> cands = {{pl.npt, pl.nps, pl.dbuf}};
  const std::array<int, 6> sig = {la, bra.one_centre ? -1 : lb, lc, ket.one_centre ? -1 : ld, maxb, maxk};
  std::vector<std::array<int, 3>> all;
  if (!diag && pl.nslab == 1 && !split) all = block_candidates(Nhb, Nb, Nk, L, cube_sz, Nhk_pad, maxpp);
  if (count) {
    *count = (int)all.size();
    return MDERI_OK;
  }
  if (tile_variant > 0) {
    if (tile_variant > (int)all.size())
      return fail(MDERI_EINVAL, "class (%d%d|%d%d): tile variant %d of %zu", la, lb, lc, ld, tile_variant, all.size());
    cands = {all[tile_variant - 1]};
  } else if (!all.empty()) {
    auto it = c->tune.find(sig);
    if (it != c->tune.end() && std::find(all.begin(), all.end(), it->second) != all.end()) cands = {it->second};
    else if (flags & MDERI_FLAG_AUTOTUNE) cands = all;
  }
  int Hb_rows = 0;
  for (auto &cd : cands) Hb_rows = std::max(Hb_rows, 16 * cd[0] * cd[1]);
  const int Hs_rows = (Hb_rows + 31) & ~31;
  const int npt = cands[0][0], nps = cands[0][1], dbuf = cands[0][2];
  const int Nhb_pad = 16 * npt * nps, Nb_pad = round16(Nb);
  const int Nk_pad = std::max(round16(Nk), 16 * pl.nct * pl.nslab);  // slabs read whole tiles
  // bank-spread order over the class's own tiles, zero rows up to Hb_rows
  std::vector<uint32_t> border = bra_row_order(Lb, S1, S2, round16(Nhb));
  while ((int)border.size() < Hb_rows) border.push_back(border[0] | kPadRow);
  const std::vector<PrimPair> &ppb = bra.pp, &ppk = ket.pp;
  const std::vector<int> &offb = bra.off, &offk = ket.off;
  mderi_status st;
  size_t scratch_used = 0;
  auto region = [&](int slot, size_t bytes, void **out) -> mderi_status {
    if (!noalloc) return ws_get(c, slot, bytes, out);
    const size_t off = scratch_used;
    scratch_used += (bytes + 255) & ~(size_t)255;
    if (scratch_used > kScratchBytes)
      return fail(MDERI_ESIZE, "class (%d%d|%d%d) with %d x %d pairs needs more than the %zu-byte scratch of the "
                  "allocation-free entry point", la, lb, lc, ld, nbra, nket, kScratchBytes);
    *out = c->scratch + off;
    return MDERI_OK;
  };
  // the call's metadata (primitive-pair lists, pair offsets, row orders and
  // the Schwarz index list) in one device region, uploaded by one copy
  struct Part {
    const void *src;
    size_t bytes, off;
  };
  Part parts[7] = {{ppb.data(), sizeof(PrimPair) * ppb.size(), 0},
                   {ppk.data(), sizeof(PrimPair) * ppk.size(), 0},
                   {offb.data(), sizeof(int) * offb.size(), 0},
                   {offk.data(), sizeof(int) * offk.size(), 0},
                   {border.data(), sizeof(uint32_t) * border.size(), 0},
                   {korder.data(), sizeof(uint32_t) * korder.size(), 0},
                   {extra_idx ? extra_idx->data() : nullptr, extra_idx ? sizeof(int) * extra_idx->size() : 0, 0}};
  size_t meta_bytes = 0;
  for (Part &pt : parts) {
    pt.off = meta_bytes;
    meta_bytes += (pt.bytes + 255) & ~(size_t)255;
  }
  void *d_meta, *d_Gb, *d_Gk, *d_Hb, *d_Hk;
  if ((st = region(WS_META, meta_bytes, &d_meta)) ||
      (st = region(WS_G_BRA, sizeof(double) * 4 * ppb.size(), &d_Gb)) ||
      (st = region(WS_G_KET, sizeof(double) * 4 * ppk.size(), &d_Gk)) ||
      (st = region(WS_H_BRA, sizeof(double) * (size_t)Hb_rows * Nb_pad * ppb.size(), &d_Hb)) ||
      (st = region(WS_H_KET, sizeof(double) * (size_t)Nhk_pad * Nk_pad * ppk.size(), &d_Hk)))
    return st;
  char *meta = (char *)d_meta;
  void *d_ppb = meta + parts[0].off, *d_ppk = meta + parts[1].off, *d_offb = meta + parts[2].off;
  void *d_offk = meta + parts[3].off, *d_border = meta + parts[4].off;
  void *d_korder = korder.empty() ? nullptr : meta + parts[5].off;
  if (extra_idx) *d_extra_idx = meta + parts[6].off;
  void *d_Hs = nullptr, *d_Hexp = nullptr, *d_Hrow = nullptr;
  if (split && ((st = region(WS_HS, sizeof(uint16_t) * slices * (size_t)Nb_pad * Hs_rows * ppb.size(), &d_Hs)) ||
                (st = region(WS_HEXP, sizeof(int) * (size_t)Nb_pad * ppb.size(), &d_Hexp)) ||
                (st = region(WS_HROW, sizeof(int) * (size_t)Hs_rows * ppb.size(), &d_Hrow))))
    return st;
  if (noalloc && meta_bytes > c->stage_cap)
    return fail(MDERI_ESIZE, "class batch metadata of %zu bytes exceeds the %zu-byte staging buffer of the "
                "allocation-free entry point", meta_bytes, c->stage_cap);
  if ((st = stage_begin(c, meta_bytes))) return st;
  for (const Part &pt : parts)
    if (pt.bytes) memcpy(c->stage_cur + pt.off, pt.src, pt.bytes);
  HIP_TRY(hipMemcpyAsync(d_meta, c->stage_cur, meta_bytes, hipMemcpyHostToDevice, s));
  if ((st = stage_end(c, s))) return st;

  PairArgs pa{};
  pa.basis = bra.b->dev;
  pa.tab = c->tab;
  pa.npp = (int)ppb.size();
  pa.pp = (const PrimPair *)d_ppb;
  pa.la = la;
  pa.lb = lb;
  pa.Nh = Nhb;
  pa.N = Nb;
  pa.Nh_pad = Hb_rows;
  pa.N_pad = Nb_pad;
  pa.ket_sign = 0;
  pa.one_centre = bra.one_centre ? 1 : 0;
  pa.deriv = 0;
  pa.split = split ? slices : 0;
  pa.Hs = (uint16_t *)d_Hs;
  pa.Hexp = (int *)d_Hexp;
  pa.Hrow = (int *)d_Hrow;
  pa.Hs_rows = Hs_rows;
  pa.order = (const uint32_t *)d_border;
  pa.G = (double *)d_Gb;
  pa.H = (double *)d_Hb;
  HIP_TRY(launch_pairs(pa, s));
  pa.basis = ket.b->dev;
  pa.npp = (int)ppk.size();
  pa.pp = (const PrimPair *)d_ppk;
  pa.la = lc;
  pa.lb = ld;
  pa.Nh = Nhk;
  pa.N = Nk;
  pa.Nh_pad = Nhk_pad;
  pa.N_pad = Nk_pad;
  pa.ket_sign = 1;
  pa.one_centre = ket.one_centre ? 1 : 0;
  pa.deriv = 0;
  pa.split = 0;
  pa.order = (const uint32_t *)d_korder;
  pa.G = (double *)d_Gk;
  pa.H = (double *)d_Hk;
  HIP_TRY(launch_pairs(pa, s));

  Eri4Args ea{};
  ea.nbra = nbra;
  ea.nket = nket;
  ea.L = L;
  ea.Nhb = Nhb;
  ea.Nhk = Nhk;
  ea.Nb = Nb;
  ea.Nk = Nk;
  ea.Nhb_pad = Nhb_pad;
  ea.Hb_rows = Hb_rows;
  ea.Nhk_pad = Nhk_pad;
  ea.Nb_pad = Nb_pad;
  ea.Nk_pad = Nk_pad;
  ea.npt = npt;
  ea.nps = nps;
  ea.nct = pl.nct;
  ea.nslab = pl.nslab;
  ea.dbuf = dbuf;
  ea.S1 = S1;
  ea.S2 = S2;
  ea.cube_sz = cube_sz;
  ea.maxpp = maxpp;
  ea.border = (const uint32_t *)d_border;
  ea.korder = (const uint32_t *)d_korder;
  ea.diag = diag;
  ea.bra_off = (const int *)d_offb;
  ea.ket_off = (const int *)d_offk;
  ea.bra_G = (const double *)d_Gb;
  ea.ket_G = (const double *)d_Gk;
  ea.bra_H = (const double *)d_Hb;
  ea.ket_H = (const double *)d_Hk;
  ea.tab = c->tab;
  ea.V = V;
  if (split) {
    ea.bra_Hs = (const uint16_t *)d_Hs;
    ea.bra_Hexp = (const int *)d_Hexp;
    ea.bra_Hrow = (const int *)d_Hrow;
    ea.Hs_rows = Hs_rows;
    ea.split = slices;
  }
  set_run_mode(ea, maxb, maxk, maxpp);
  if (cands.size() > 1) {
    // autotune: time each variant on this batch (the second of two runs)
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    std::array<int, 3> bestc = cands[0];
    for (auto &cd : cands) {
      Eri4Args t = ea;
      t.npt = cd[0];
      t.nps = cd[1];
      t.dbuf = cd[2];
      t.Nhb_pad = 16 * cd[0] * cd[1];
      set_run_mode(t, maxb, maxk, maxpp);
      float ms = 0.0f;
      for (int rep = 0; rep < 2; ++rep) {
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(launch_eri4(t, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best) {
        best = ms;
        bestc = cd;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tune[sig] = bestc;
    ea.npt = bestc[0];
    ea.nps = bestc[1];
    ea.dbuf = bestc[2];
    ea.Nhb_pad = 16 * bestc[0] * bestc[1];
    set_run_mode(ea, maxb, maxk, maxpp);
  }
  if (noalloc) {  // no timing events (creating them could allocate)
    HIP_TRY(launch_eri4(ea, s));
    return MDERI_OK;
  }
  return launch_eri4_timed(c, ea, s);
}

// Validates single shells of one l and expands them into primitives.
mderi_status expand_shells(const mderi_basis *b, int n, const int32_t *idx, const char *what, int *l, Side &side) {
  if (n <= 0) return fail(MDERI_EINVAL, "%s: need at least one shell (got %d)", what, n);
  if (!idx) return fail(MDERI_EINVAL, "%s: NULL shell list", what);
  side.pp.clear();
  side.off.assign(1, 0);
  for (int i = 0; i < n; ++i) {
    const int s0 = idx[i];
    if (s0 < 0 || s0 >= b->nshell) return fail(MDERI_EINVAL, "%s: shell %d = %d out of range [0,%d)", what, i, s0, b->nshell);
    if (i == 0) *l = b->l[s0];
    else if (b->l[s0] != *l)
      return fail(MDERI_EINVAL, "%s: shell %d has l=%d but the batch has l=%d", what, i, b->l[s0], *l);
    for (int k = 0; k < b->K[s0]; ++k) side.pp.push_back(PrimPair{s0, s0, b->poff[s0] + k, b->poff[s0] + k});
    side.off.push_back((int)side.pp.size());
  }
  return MDERI_OK;
}

}  // namespace

extern "C" mderi_status mderi_eri4(mderi_ctx_t c, mderi_basis_t b, int nbra, const int32_t *bra, int nket,
                                   const int32_t *ket, double *V, size_t V_elems, const mderi_opts *opts,
                                   void *stream) {
  if (!c || !b) return fail(MDERI_EINVAL, "mderi_eri4: NULL context or basis");
  if (b->ctx != c) return fail(MDERI_EINVAL, "mderi_eri4: basis belongs to another context");
  const int precision = opts ? opts->precision : 0;
  if (precision != MDERI_FP64 && precision != MDERI_SPLIT_BF16)
    return fail(MDERI_EUNSUPPORTED, "mderi_eri4: precision %d", precision);
  const int slices = (opts && opts->split_slices) ? opts->split_slices : kSplitDefault;
  if (precision == MDERI_SPLIT_BF16 && (slices < kSplitMin || slices > kSplitMax))
    return fail(MDERI_EINVAL, "mderi_eri4: split_slices %d outside [%d,%d]", slices, kSplitMin, kSplitMax);
  Side sb{b, 0, 0, false, {}, {}}, sk{b, 0, 0, false, {}, {}};
  mderi_status st;
  if ((st = expand_pairs(b, nbra, bra, "bra", &sb.la, &sb.lb, sb.pp, sb.off)) != MDERI_OK) return st;
  if ((st = expand_pairs(b, nket, ket, "ket", &sk.la, &sk.lb, sk.pp, sk.off)) != MDERI_OK) return st;
  const size_t need = (size_t)nbra * nsph(sb.la) * nsph(sb.lb) * nsph(sk.la) * nsph(sk.lb) * nket;
  if (!V) return fail(MDERI_EINVAL, "mderi_eri4: NULL output");
  if (V_elems < need) return fail(MDERI_ESIZE, "mderi_eri4: output holds %zu doubles, needs %zu", V_elems, need);
  const int flags = opts ? opts->flags : 0;
  if (flags & ~MDERI_FLAG_AUTOTUNE) return fail(MDERI_EINVAL, "mderi_eri4: unsupported flags 0x%x", flags);
  const int variant = opts ? opts->tile_variant : 0;
  if (variant < 0 || (variant > 0 && precision != MDERI_FP64))
    return fail(MDERI_EINVAL, "mderi_eri4: tile_variant %d (FP64 batches only, >= 0)", variant);
  HIP_TRY(hipSetDevice(c->device));
  return run_class_batch(c, sb, sk, 0, V, nullptr, nullptr, (hipStream_t)stream, flags, precision, slices, false,
                         variant);
}

extern "C" mderi_status mderi_eri4_tile_variants(mderi_ctx_t c, mderi_basis_t b, int nbra, const int32_t *bra,
                                                 int nket, const int32_t *ket, int *count) {
  if (!c || !b) return fail(MDERI_EINVAL, "mderi_eri4_tile_variants: NULL context or basis");
  if (b->ctx != c) return fail(MDERI_EINVAL, "mderi_eri4_tile_variants: basis belongs to another context");
  if (!count) return fail(MDERI_EINVAL, "mderi_eri4_tile_variants: NULL count");
  Side sb{b, 0, 0, false, {}, {}}, sk{b, 0, 0, false, {}, {}};
  mderi_status st;
  if ((st = expand_pairs(b, nbra, bra, "bra", &sb.la, &sb.lb, sb.pp, sb.off)) != MDERI_OK) return st;
  if ((st = expand_pairs(b, nket, ket, "ket", &sk.la, &sk.lb, sk.pp, sk.off)) != MDERI_OK) return st;
  return run_class_batch(c, sb, sk, 0, nullptr, nullptr, nullptr, nullptr, 0, MDERI_FP64, kSplitDefault, false, 0,
                         count);
}

extern "C" mderi_status mderi_eri4_noalloc(mderi_ctx_t c, mderi_basis_t b, int nbra, const int32_t *bra, int nket,
                                           const int32_t *ket, double *V, size_t V_elems, const mderi_opts *opts,
                                           void *stream) {
  if (!c || !b) return fail(MDERI_EINVAL, "mderi_eri4_noalloc: NULL context or basis");
  if (b->ctx != c) return fail(MDERI_EINVAL, "mderi_eri4_noalloc: basis belongs to another context");
  if (opts && opts->precision != MDERI_FP64)
    return fail(MDERI_EUNSUPPORTED, "mderi_eri4_noalloc: precision %d (FP64 only)", opts->precision);
  if (opts && opts->flags) return fail(MDERI_EINVAL, "mderi_eri4_noalloc: flags 0x%x (none supported)", opts->flags);
  Side sb{b, 0, 0, false, {}, {}}, sk{b, 0, 0, false, {}, {}};
  mderi_status st;
  if ((st = expand_pairs(b, nbra, bra, "bra", &sb.la, &sb.lb, sb.pp, sb.off)) != MDERI_OK) return st;
  if ((st = expand_pairs(b, nket, ket, "ket", &sk.la, &sk.lb, sk.pp, sk.off)) != MDERI_OK) return st;
  const size_t need = (size_t)nbra * nsph(sb.la) * nsph(sb.lb) * nsph(sk.la) * nsph(sk.lb) * nket;
  if (!V) return fail(MDERI_EINVAL, "mderi_eri4_noalloc: NULL output");
  if (V_elems < need)
    return fail(MDERI_ESIZE, "mderi_eri4_noalloc: output holds %zu doubles, needs %zu", V_elems, need);
  HIP_TRY(hipSetDevice(c->device));
  return run_class_batch(c, sb, sk, 0, V, nullptr, nullptr, (hipStream_t)stream, 0, MDERI_FP64, kSplitDefault, true);
}

extern "C" mderi_status mderi_eri3(mderi_ctx_t c, mderi_basis_t b, mderi_basis_t aux, int npair, const int32_t *pairs,
                                   int naux, const int32_t *auxidx, double *V, size_t V_elems, const mderi_opts *opts,
                                   void *stream) {
  if (!c || !b || !aux) return fail(MDERI_EINVAL, "mderi_eri3: NULL context or basis");
  if (b->ctx != c || aux->ctx != c) return fail(MDERI_EINVAL, "mderi_eri3: basis belongs to another context");
  if (opts && opts->precision != 0) return fail(MDERI_EUNSUPPORTED, "mderi_eri3: precision %d", opts->precision);
  Side sb{b, 0, 0, false, {}, {}}, sk{aux, 0, 0, true, {}, {}};
  mderi_status st;
  if ((st = expand_pairs(b, npair, pairs, "pairs", &sb.la, &sb.lb, sb.pp, sb.off)) != MDERI_OK) return st;
  if ((st = expand_shells(aux, naux, auxidx, "aux", &sk.la, sk)) != MDERI_OK) return st;
  const size_t need = (size_t)npair * nsph(sb.la) * nsph(sb.lb) * nsph(sk.la) * naux;
  if (!V) return fail(MDERI_EINVAL, "mderi_eri3: NULL output");
  if (V_elems < need) return fail(MDERI_ESIZE, "mderi_eri3: output holds %zu doubles, needs %zu", V_elems, need);
  HIP_TRY(hipSetDevice(c->device));
  return run_class_batch(c, sb, sk, 0, V, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" mderi_status mderi_eri2(mderi_ctx_t c, mderi_basis_t b, int na, const int32_t *shells_a, int nc,
                                   const int32_t *shells_c, double *V, size_t V_elems, const mderi_opts *opts,
                                   void *stream) {
  if (!c || !b) return fail(MDERI_EINVAL, "mderi_eri2: NULL context or basis");
  if (b->ctx != c) return fail(MDERI_EINVAL, "mderi_eri2: basis belongs to another context");
  if (opts && opts->precision != 0) return fail(MDERI_EUNSUPPORTED, "mderi_eri2: precision %d", opts->precision);
  // both sides single shells: the 1-centre Hermite expansion on the bra as on
  // the ket of the 3-centre integrals
  Side sa{b, 0, 0, true, {}, {}}, sc{b, 0, 0, true, {}, {}};
  mderi_status st;
  if ((st = expand_shells(b, na, shells_a, "shells_a", &sa.la, sa)) != MDERI_OK) return st;
  if ((st = expand_shells(b, nc, shells_c, "shells_c", &sc.la, sc)) != MDERI_OK) return st;
  const size_t need = (size_t)na * nsph(sa.la) * nsph(sc.la) * nc;
  if (!V) return fail(MDERI_EINVAL, "mderi_eri2: NULL output");
  if (V_elems < need) return fail(MDERI_ESIZE, "mderi_eri2: output holds %zu doubles, needs %zu", V_elems, need);
  HIP_TRY(hipSetDevice(c->device));
  return run_class_batch(c, sa, sc, 0, V, nullptr, nullptr, (hipStream_t)stream,
                         (opts && (opts->flags & MDERI_FLAG_AUTOTUNE)) ? MDERI_FLAG_AUTOTUNE : 0);
}

extern "C" mderi_status mderi_schwarz(mderi_ctx_t c, mderi_basis_t b, int npair, const int32_t *pairs, double *Q,
                                      void *stream) {
  if (!c || !b) return fail(MDERI_EINVAL, "mderi_schwarz: NULL context or basis");
  if (b->ctx != c) return fail(MDERI_EINVAL, "mderi_schwarz: basis belongs to another context");
  if (npair <= 0 || !pairs) return fail(MDERI_EINVAL, "mderi_schwarz: need a non-empty pair list");
  if (!Q) return fail(MDERI_EINVAL, "mderi_schwarz: NULL output");
  for (int i = 0; i < npair; ++i)
    if (pairs[2 * i] < 0 || pairs[2 * i] >= b->nshell || pairs[2 * i + 1] < 0 || pairs[2 * i + 1] >= b->nshell)
      return fail(MDERI_EINVAL, "mderi_schwarz: pair %d = (%d,%d) out of range", i, pairs[2 * i], pairs[2 * i + 1]);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  // group by class (la, lb)
  std::vector<std::vector<int>> groups((kLmax + 1) * (kLmax + 1));
  for (int i = 0; i < npair; ++i) groups[b->l[pairs[2 * i]] * (kLmax + 1) + b->l[pairs[2 * i + 1]]].push_back(i);
  mderi_status st;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const std::vector<int> &grp = groups[gi];
    if (grp.empty()) continue;
    std::vector<int32_t> sub(2 * grp.size());
    for (size_t k = 0; k < grp.size(); ++k) {
      sub[2 * k] = pairs[2 * grp[k]];
      sub[2 * k + 1] = pairs[2 * grp[k] + 1];
    }
    Side sd{b, 0, 0, false, {}, {}};
    if ((st = expand_pairs(b, (int)grp.size(), sub.data(), "pairs", &sd.la, &sd.lb, sd.pp, sd.off)) != MDERI_OK)
      return st;
    const int Nab = nsph(sd.la) * nsph(sd.lb);
    void *d_diag, *d_idx = nullptr;
    if ((st = ws_get(c, WS_DIAG, sizeof(double) * grp.size() * Nab, &d_diag))) return st;
    if ((st = run_class_batch(c, sd, sd, 1, (double *)d_diag, &grp, &d_idx, s))) return st;
    HIP_TRY(launch_schwarz_reduce((int)grp.size(), Nab, (const double *)d_diag, (const int *)d_idx, Q, s));
  }
  return MDERI_OK;
}

namespace {

// Canonical shell pairs (l_i > l_j, or l_i == l_j and i >= j) whose Schwarz
// factor passes Q_ij Q_max >= tau, grouped by class (l_i, l_j) and expanded
// into primitive pairs.  The selection runs on the host: the first call for a
// (basis upload, geometry, tau) key synchronises the stream once; later calls
// with the same key take the context's cached copy and do not wait.
struct PairSets {
  std::vector<int32_t> pairs;          // all canonical pairs [np][2]
  std::vector<double> q;               // their Schwarz factors
  std::vector<std::vector<int>> cls;   // significant pairs per class
  std::vector<Side> sides;             // their primitive expansion
};

mderi_status select_pairs_uncached(mderi_ctx *c, mderi_basis *b, double tau, hipStream_t s, PairSets &ps) {
  for (int i = 0; i < b->nshell; ++i)
    for (int j = 0; j < b->nshell; ++j)
      if (b->l[i] > b->l[j] || (b->l[i] == b->l[j] && i >= j)) {
        ps.pairs.push_back(i);
        ps.pairs.push_back(j);
      }
  const int np = (int)ps.pairs.size() / 2;
  mderi_status st;
  void *d_q;
  if ((st = ws_get(c, WS_QALL, sizeof(double) * np, &d_q))) return st;
  if ((st = mderi_schwarz(c, b, np, ps.pairs.data(), (double *)d_q, s))) return st;
  ps.q.assign(np, 0.0);
  HIP_TRY(hipMemcpyAsync(ps.q.data(), d_q, sizeof(double) * np, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double qmax = 0.0;
  for (double x : ps.q) qmax = std::max(qmax, x);
  const int ncls = (kLmax + 1) * (kLmax + 1);
  ps.cls.assign(ncls, {});
  for (int p = 0; p < np; ++p)
    if (ps.q[p] * qmax >= tau) ps.cls[b->l[ps.pairs[2 * p]] * (kLmax + 1) + b->l[ps.pairs[2 * p + 1]]].push_back(p);
  // decreasing Q inside each class: the partners that pass Q_i Q_k >= tau
  // are then a prefix of the class's list
  for (auto &cl : ps.cls)
    std::stable_sort(cl.begin(), cl.end(), [&](int x, int y) { return ps.q[x] > ps.q[y]; });
  ps.sides.assign(ncls, Side{b, 0, 0, false, {}, {}});
  for (int ci = 0; ci < ncls; ++ci) {
    if (ps.cls[ci].empty()) continue;
    std::vector<int32_t> sub;
    for (int p : ps.cls[ci]) {
      sub.push_back(ps.pairs[2 * p]);
      sub.push_back(ps.pairs[2 * p + 1]);
    }
    Side &sd = ps.sides[ci];
    if ((st = expand_pairs(b, (int)ps.cls[ci].size(), sub.data(), "pairs", &sd.la, &sd.lb, sd.pp, sd.off))) return st;
  }
  return MDERI_OK;
}

mderi_status select_pairs(mderi_ctx *c, mderi_basis *b, double tau, hipStream_t s,
                          std::shared_ptr<const PairSets> &out) {
  auto &pc = c->pair_cache;
  for (size_t i = 0; i < pc.size(); ++i)
    if (pc[i].serial == b->serial && pc[i].geom == b->geom && pc[i].tau == tau) {
      out = pc[i].ps;
      if (i + 1 != pc.size()) std::rotate(pc.begin() + i, pc.begin() + i + 1, pc.end());
      return MDERI_OK;
    }
  auto ps = std::make_shared<PairSets>();
  mderi_status st;
  if ((st = select_pairs_uncached(c, b, tau, s, *ps))) return st;
  if (pc.size() >= kPairCacheKeys) pc.erase(pc.begin());
  pc.push_back({b->serial, b->geom, tau, ps});
  out = ps;
  return MDERI_OK;
}

void drop_pair_selections(mderi_basis *b) {
  auto &pc = b->ctx->pair_cache;
  pc.erase(std::remove_if(pc.begin(), pc.end(), [&](const mderi_ctx::PairCacheEntry &e) { return e.serial == b->serial; }),
           pc.end());
}

mderi_status check_density(const char *fn, mderi_ctx *c, mderi_basis *b, const double *D, int nao,
                           const mderi_opts *opts) {
  if (!c || !b) return fail(MDERI_EINVAL, "%s: NULL context or basis", fn);
  if (b->ctx != c) return fail(MDERI_EINVAL, "%s: basis belongs to another context", fn);
  if (!D) return fail(MDERI_EINVAL, "%s: NULL density", fn);
  if (nao != b->nao) return fail(MDERI_EINVAL, "%s: nao=%d but the basis has %d AOs", fn, nao, b->nao);
  if (opts && opts->precision != 0) return fail(MDERI_EUNSUPPORTED, "%s: precision %d", fn, opts->precision);
  if (opts && opts->deterministic != 0 && opts->deterministic != 1)
    return fail(MDERI_EINVAL, "%s: deterministic %d (0 or 1)", fn, opts->deterministic);
  return MDERI_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// task lists: mixed-class 3-centre batches in persistent launches
// ---------------------------------------------------------------------------
constexpr int kSideStreams = 4;  // one per hardware queue of the process

struct TaskGroup {
  int npt, Lmax, waves, grid, ntask;
  size_t lds;
  const Eri4Args *d_blocks;
  const int2 *d_tasks;
};

struct TaskPlan {
  uint64_t key = 0;
  int flags = 0;
  void *dmem = nullptr;  // one device allocation holding every array of the plan
  std::vector<PairArgs> pairs;  // pair-data launches (bra classes, then aux l)
  std::vector<TaskGroup> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // fork/join events: the groups run concurrently on the context's side
  // streams (a captured graph keeps them as parallel branches)
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

void free_plan(TaskPlan *p) {
  if (!p) return;
  if (p->fork) (void)hipEventDestroy(p->fork);
  for (hipEvent_t e : p->join) (void)hipEventDestroy(e);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
}

namespace {

uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
  const unsigned char *d = (const unsigned char *)data;
  for (size_t i = 0; i < n; ++i) h = (h ^ d[i]) * 1099511628211ull;
  return h;
}

// Host image of the plan's device arrays: every array is appended at a
// 256-byte aligned offset; device pointers are base + offset once the single
// allocation exists.
// Layout of one device allocation: regions of 256-byte aligned offsets.
// Regions added with host data are kept in `bytes` (zeros in between) for
// one upload of the leading bytes.size() bytes; regions the device fills
// (src == nullptr) only advance `size`, so large pair-data regions cost no
// host memory.
struct Image {
  std::vector<char> bytes;
  size_t size = 0;
  size_t add(const void *src, size_t n) {
    const size_t off = (size + 255) & ~(size_t)255;
    size = off + ((n + 255) & ~(size_t)255);
    if (src) {
      bytes.resize(size, 0);
      if (n) memcpy(bytes.data() + off, src, n);
    }
    return off;
  }
};

// Candidate (npt, nps, dbuf) plans of a block: every row split with at most
// 6 tiles per wave that fits the wave and LDS limits; the first is the
// default (fewest waves).
std::vector<std::array<int, 3>> block_candidates(int Nhb, int Nb, int Nk, int L, int cube_sz, int Nhk_pad,
                                                 int maxpp) {
  std::vector<std::array<int, 3>> out;
  Eri4Plan pl{};
  if (!eri4_plan(Nhb, Nb, Nk, L, cube_sz, Nhk_pad, maxpp, false, &pl)) return out;
  const int dbuf = pl.dbuf;
  out.push_back({pl.npt, pl.nps, pl.dbuf});
  const int need = (Nhb + 15) / 16, nct = (Nk + 15) / 16;
  const int tiles[] = {1, 2, 3, 4, 6};
  for (int parts = 1; parts <= 4; ++parts) {
    const int per = (need + parts - 1) / parts;
    int t = 0;
    for (int x : tiles)
      if (x >= per) {
        t = x;
        break;
      }
    if (!t || nct * parts + 1 > 16) continue;
    for (int db = 1; db >= 0; --db) {
      if (db && !dbuf) continue;  // double buffering does not fit
      const std::array<int, 3> cand = {t, parts, db};
      if (std::find(out.begin(), out.end(), cand) == out.end()) out.push_back(cand);
    }
  }
  return out;
}

size_t block_lds(const Eri4Args &a) { return eri4_lds_bytes(a); }

int group_grid(size_t lds, int waves, long ntask, int occ = 4) {
  const long per_cu_lds = lds ? (long)(160 * 1024 / lds) : 16;
  const long per_cu_waves = 4 * occ / waves;  // occ waves per SIMD (128 VGPRs per lane: 4)
  long per_cu = std::max(1L, std::min(per_cu_lds, per_cu_waves));
  long g = 256 * per_cu;
  return (int)std::max(1L, std::min(g, ntask));
}

// Task-list launches of a plan: one per kernel shape, each on its own side
// stream after a fork from s and joined back into s, so that small groups
// fill the chip together instead of one after another.
mderi_status launch_groups(mderi_ctx *c, TaskPlan *p, hipStream_t s) {
  if (p->groups.size() == 1) {
    const TaskGroup &g = p->groups[0];
    HIP_TRY(launch_eri4_tasks(g.d_blocks, g.d_tasks, g.ntask, g.npt, g.Lmax, g.waves, g.lds, g.grid, s));
    return MDERI_OK;
  }
  for (int i = (int)c->side.size(); i < kSideStreams; ++i) {
    hipStream_t x;
    HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    c->side.push_back(x);
  }
  if (!p->fork) {
    HIP_TRY(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    p->join.resize(p->groups.size(), nullptr);
    for (auto &e : p->join) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(p->fork, s));
  for (size_t i = 0; i < p->groups.size(); ++i) {
    const TaskGroup &g = p->groups[i];
    hipStream_t x = c->side[i % kSideStreams];
    HIP_TRY(hipStreamWaitEvent(x, p->fork, 0));
    HIP_TRY(launch_eri4_tasks(g.d_blocks, g.d_tasks, g.ntask, g.npt, g.Lmax, g.waves, g.lds, g.grid, x));
    HIP_TRY(hipEventRecord(p->join[i], x));
  }
  for (hipEvent_t e : p->join) HIP_TRY(hipStreamWaitEvent(s, e, 0));
  return MDERI_OK;
}

mderi_status launch_plan(mderi_ctx *c, TaskPlan *p, hipStream_t s) {
  for (const PairArgs &pa : p->pairs) HIP_TRY(launch_pairs(pa, s));
  return launch_groups(c, p, s);
}

}  // namespace

extern "C" mderi_status mderi_eri3_batch(mderi_ctx_t c, mderi_basis_t b, mderi_basis_t aux, int npair,
                                         const int32_t *pairs, int naux, const int32_t *auxidx, double *V,
                                         size_t V_elems, const mderi_opts *opts, void *stream) {
  if (!c || !b || !aux) return fail(MDERI_EINVAL, "mderi_eri3_batch: NULL context or basis");
  if (b->ctx != c || aux->ctx != c) return fail(MDERI_EINVAL, "mderi_eri3_batch: basis belongs to another context");
  if (opts && opts->precision != 0) return fail(MDERI_EUNSUPPORTED, "mderi_eri3_batch: precision %d", opts->precision);
  if (npair <= 0 || naux <= 0 || !pairs || !auxidx)
    return fail(MDERI_EINVAL, "mderi_eri3_batch: need non-empty pair and aux lists");
  if (!V) return fail(MDERI_EINVAL, "mderi_eri3_batch: NULL output");
  const int flags = opts ? opts->flags : 0;
  if (flags & ~(MDERI_FLAG_GRAPH | MDERI_FLAG_AUTOTUNE))
    return fail(MDERI_EINVAL, "mderi_eri3_batch: unknown flags 0x%x", flags);
  for (int i = 0; i < npair; ++i)
    if (pairs[2 * i] < 0 || pairs[2 * i] >= b->nshell || pairs[2 * i + 1] < 0 || pairs[2 * i + 1] >= b->nshell)
      return fail(MDERI_EINVAL, "mderi_eri3_batch: pair %d = (%d,%d) out of range [0,%d)", i, pairs[2 * i],
                  pairs[2 * i + 1], b->nshell);
  for (int k = 0; k < naux; ++k)
    if (auxidx[k] < 0 || auxidx[k] >= aux->nshell)
      return fail(MDERI_EINVAL, "mderi_eri3_batch: aux %d = %d out of range [0,%d)", k, auxidx[k], aux->nshell);
  // output geometry: rows = AO pairs in list order, columns = aux AOs in list order
  std::vector<long> rowoff(npair), coloff(naux);
  long nrow = 0, ncol = 0;
  for (int i = 0; i < npair; ++i) {
    rowoff[i] = nrow;
    nrow += (long)nsph(b->l[pairs[2 * i]]) * nsph(b->l[pairs[2 * i + 1]]);
  }
  for (int k = 0; k < naux; ++k) {
    coloff[k] = ncol;
    ncol += nsph(aux->l[auxidx[k]]);
  }
  if (V_elems < (size_t)nrow * (size_t)ncol)
    return fail(MDERI_ESIZE, "mderi_eri3_batch: output holds %zu doubles, needs %ld", V_elems, nrow * ncol);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;

  uint64_t key = 1469598103934665603ull;
  key = fnv1a(key, &b->serial, sizeof(b->serial));
  key = fnv1a(key, &aux->serial, sizeof(aux->serial));
  key = fnv1a(key, &npair, sizeof(npair));
  key = fnv1a(key, pairs, sizeof(int32_t) * 2 * (size_t)npair);
  key = fnv1a(key, &naux, sizeof(naux));
  key = fnv1a(key, auxidx, sizeof(int32_t) * (size_t)naux);
  key = fnv1a(key, &V, sizeof(V));
  key = fnv1a(key, &flags, sizeof(flags));
  for (size_t i = 0; i < c->plans.size(); ++i) {
    TaskPlan *p = c->plans[i];
    if (p->key != key) continue;
    c->plans.erase(c->plans.begin() + i);
    c->plans.push_back(p);  // most recently used last
    if (p->exec) {
      HIP_TRY(hipGraphLaunch(p->exec, s));
      return MDERI_OK;
    }
    return launch_plan(c, p, s);
  }

  // ---- build the plan ----
  // classes: bra (la, lb) groups of pairs; aux l groups of shells
  std::map<std::pair<int, int>, std::vector<int>> bcls;
  std::map<int, std::vector<int>> acls;
  for (int i = 0; i < npair; ++i) bcls[{b->l[pairs[2 * i]], b->l[pairs[2 * i + 1]]}].push_back(i);
  for (int k = 0; k < naux; ++k) acls[aux->l[auxidx[k]]].push_back(k);
  const int lPmax = acls.rbegin()->first;
  mderi_status st;
  Image img;
  struct SideData {
    int la, lb, Nh, N, Nh_pad, N_pad, S1, S2, npp, maxpp;
    size_t o_pp, o_off, o_G, o_H, o_order, o_rows;
    std::vector<int> off;
  };
  // aux (1-centre ket) sides, one per l
  std::map<int, SideData> aside;
  for (auto &kv : acls) {
    const int l = kv.first;
    std::vector<PrimPair> pp;
    std::vector<int> off(1, 0);
    std::vector<long> cols;
    for (int k : kv.second) {
      const int sh = auxidx[k];
      for (int q = 0; q < aux->K[sh]; ++q) pp.push_back(PrimPair{sh, sh, aux->poff[sh] + q, aux->poff[sh] + q});
      off.push_back((int)pp.size());
      cols.push_back(coloff[k]);
    }
    std::vector<uint32_t> ko = top_degree_rows(l);
    SideData d{};
    d.la = l;
    d.lb = 0;
    d.Nh = (l + 1) * (l + 2) / 2;
    d.N = nsph(l);
    d.Nh_pad = (int)ko.size();
    d.N_pad = round16(d.N);
    d.npp = (int)pp.size();
    d.maxpp = 0;
    for (size_t i = 0; i + 1 < off.size(); ++i) d.maxpp = std::max(d.maxpp, off[i + 1] - off[i]);
    d.o_pp = img.add(pp.data(), sizeof(PrimPair) * pp.size());
    d.o_off = img.add(off.data(), sizeof(int) * off.size());
    d.o_G = img.add(nullptr, sizeof(double) * 4 * pp.size());
    d.o_H = img.add(nullptr, sizeof(double) * (size_t)d.Nh_pad * d.N_pad * pp.size());
    d.o_order = img.add(ko.data(), sizeof(uint32_t) * ko.size());
    d.o_rows = img.add(cols.data(), sizeof(long) * cols.size());
    d.off = off;
    aside[l] = d;
  }
  // bra sides, one per class; strides fit the largest L the class meets
  std::map<std::pair<int, int>, SideData> bside;
  struct BlockPlan {
    std::pair<int, int> bc;
    int l;
    Eri4Args a;
    std::vector<std::array<int, 3>> cands;
    std::array<int, 6> sig;
  };
  std::vector<BlockPlan> blocks;
  for (auto &kv : bcls) {
    const int la = kv.first.first, lb = kv.first.second, Lb = la + lb;
    std::vector<PrimPair> pp;
    std::vector<int> off(1, 0);
    std::vector<long> rows;
    int maxb = 0;
    for (int i : kv.second) {
      const int s0 = pairs[2 * i], s1 = pairs[2 * i + 1];
      for (int ka = 0; ka < b->K[s0]; ++ka)
        for (int kb = 0; kb < b->K[s1]; ++kb) pp.push_back(PrimPair{s0, s1, b->poff[s0] + ka, b->poff[s1] + kb});
      off.push_back((int)pp.size());
      maxb = std::max(maxb, off.back() - off[off.size() - 2]);
      rows.push_back(rowoff[i]);
    }
    SideData d{};
    d.la = la;
    d.lb = lb;
    d.Nh = ntil(Lb);
    d.N = nsph(la) * nsph(lb);
    d.N_pad = round16(d.N);
    choose_cube(Lb + lPmax, Lb, &d.S1, &d.S2);
    d.npp = (int)pp.size();
    d.maxpp = maxb;
    // blocks of this class and their candidate tiles
    int nh_pad = round16(d.Nh);
    for (auto &akv : aside) {
      const SideData &ad = akv.second;
      const int L = Lb + ad.la;
      BlockPlan bp;
      bp.bc = kv.first;
      bp.l = ad.la;
      Eri4Args &a = bp.a;
      a = Eri4Args{};
      a.nbra = (int)kv.second.size();
      a.nket = (int)acls[ad.la].size();
      a.L = L;
      a.Nhb = d.Nh;
      a.Nhk = ad.Nh;
      a.Nb = d.N;
      a.Nk = ad.N;
      a.Nb_pad = d.N_pad;
      a.Nhk_pad = ad.Nh_pad;
      a.Nk_pad = ad.N_pad;
      a.nct = ad.N_pad / 16;
      a.nslab = 1;
      choose_cube(L, Lb, &a.S1, &a.S2);  // the block's own L (small cubes for small l_P)
      a.cube_sz = (L * a.S1 + 2) & ~1;
      a.maxpp = maxb + ad.maxpp;
      a.ld = nrow;
      bp.cands = block_candidates(a.Nhb, a.Nb, a.Nk, L, a.cube_sz, a.Nhk_pad, a.maxpp);
      if (bp.cands.empty())
        return fail(MDERI_EUNSUPPORTED, "mderi_eri3_batch: class (%d%d|%d) is beyond the fused kernel's tiles", la, lb,
                    ad.la);
      int kb = 0, kk = 0;
      for (int i : kv.second) kb = std::max(kb, b->K[pairs[2 * i]] * b->K[pairs[2 * i + 1]]);
      for (int k : acls[ad.la]) kk = std::max(kk, aux->K[auxidx[k]]);
      bp.sig = {la, lb, ad.la, -1, kb, kk};
      auto it = c->tune.find(bp.sig);
      if (it != c->tune.end() &&
          std::find(bp.cands.begin(), bp.cands.end(), it->second) != bp.cands.end()) {
        bp.cands = {it->second};
      } else if (!(flags & MDERI_FLAG_AUTOTUNE)) {
        bp.cands.resize(1);
      }
      for (auto &cd : bp.cands) nh_pad = std::max(nh_pad, 16 * cd[0] * cd[1]);
      blocks.push_back(bp);
    }
    d.Nh_pad = nh_pad;
    // bank-spread row order over the class's own tiles, then zero padding rows
    std::vector<uint32_t> order = bra_row_order(Lb, d.S1, d.S2, round16(d.Nh));
    while ((int)order.size() < nh_pad) order.push_back(order[0] | kPadRow);
    d.o_pp = img.add(pp.data(), sizeof(PrimPair) * pp.size());
    d.o_off = img.add(off.data(), sizeof(int) * off.size());
    d.o_G = img.add(nullptr, sizeof(double) * 4 * pp.size());
    d.o_H = img.add(nullptr, sizeof(double) * (size_t)nh_pad * d.N_pad * pp.size());
    d.o_order = img.add(order.data(), sizeof(uint32_t) * order.size());
    d.o_rows = img.add(rows.data(), sizeof(long) * rows.size());
    d.off = off;
    bside[kv.first] = d;
  }
  // space for block descriptors and task lists (filled after tuning)
  const size_t o_blocks = img.add(nullptr, sizeof(Eri4Args) * blocks.size());
  long ntask_all = 0;
  for (auto &bp : blocks) ntask_all += (long)bp.a.nbra * bp.a.nket;
  if (ntask_all > 0x7fffffffL) return fail(MDERI_EUNSUPPORTED, "mderi_eri3_batch: %ld triplets is too many", ntask_all);
  const size_t o_tasks = img.add(nullptr, sizeof(int2) * (size_t)ntask_all);

  TaskPlan *plan = new TaskPlan;
  plan->key = key;
  plan->flags = flags;
  if (hipMalloc(&plan->dmem, img.size) != hipSuccess) {
    (void)hipGetLastError();
    delete plan;
    return fail(MDERI_ENOMEM, "mderi_eri3_batch: plan of %zu bytes could not be allocated", img.size);
  }
  char *base = (char *)plan->dmem;
  auto dev = [&](size_t off) { return (void *)(base + off); };
  // fill descriptors (pointers are final now)
  for (auto &bp : blocks) {
    const SideData &bd = bside[bp.bc], &ad = aside[bp.l];
    Eri4Args &a = bp.a;
    a.Hb_rows = bd.Nh_pad;
    a.bra_off = (const int *)dev(bd.o_off);
    a.ket_off = (const int *)dev(ad.o_off);
    a.bra_G = (const double *)dev(bd.o_G);
    a.ket_G = (const double *)dev(ad.o_G);
    a.bra_H = (const double *)dev(bd.o_H);
    a.ket_H = (const double *)dev(ad.o_H);
    a.border = (const uint32_t *)dev(bd.o_order);
    a.korder = (const uint32_t *)dev(ad.o_order);
    a.orow = (const long *)dev(bd.o_rows);
    a.ocol = (const long *)dev(ad.o_rows);
    a.tab = c->tab;
    a.V = V;
  }
  // pair-data launches
  auto pair_args = [&](const SideData &d, const mderi_basis *bb, bool ket) {
    PairArgs pa{};
    pa.basis = bb->dev;
    pa.tab = c->tab;
    pa.npp = d.npp;
    pa.pp = (const PrimPair *)dev(d.o_pp);
    pa.la = d.la;
    pa.lb = d.lb;
    pa.Nh = d.Nh;
    pa.N = d.N;
    pa.Nh_pad = d.Nh_pad;
    pa.N_pad = d.N_pad;
    pa.ket_sign = ket ? 1 : 0;
    pa.one_centre = ket ? 1 : 0;
    pa.deriv = 0;
    pa.order = (const uint32_t *)dev(d.o_order);
    pa.G = (double *)dev(d.o_G);
    pa.H = (double *)dev(d.o_H);
    return pa;
  };
  for (auto &kv : bside) plan->pairs.push_back(pair_args(kv.second, b, false));
  for (auto &kv : aside) plan->pairs.push_back(pair_args(kv.second, aux, true));
  // upload the host-written regions (pair lists, offsets, row orders; the
  // descriptors and tasks follow, the pair data is written by its kernels)
  if (hipMemcpy(base, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(plan);
    return fail(MDERI_EDEVICE, "mderi_eri3_batch: plan upload failed");
  }
  for (const PairArgs &pa : plan->pairs)
    if (launch_pairs(pa, s) != hipSuccess) {
      free_plan(plan);
      return fail(MDERI_EDEVICE, "mderi_eri3_batch: pair-data launch failed");
    }
  // per-block task lists (quartet index ij + nbra kl), cost for ordering
  auto block_cost = [&](const BlockPlan &bp) {
    const Eri4Args &a = bp.a;
    return (double)a.Nhb * a.Nhk * a.Nk + (double)a.Nb * a.Nhb * a.Nk + (double)(a.L + 1) * (a.L + 2) * (a.L + 3) / 6;
  };
  // autotune: time each candidate of an untuned block alone
  if (flags & MDERI_FLAG_AUTOTUNE) {
    std::vector<Eri4Args> one(1);
    std::vector<int2> tk;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    for (size_t bi = 0; bi < blocks.size(); ++bi) {
      BlockPlan &bp = blocks[bi];
      if (bp.cands.size() <= 1) continue;
      const int nq = bp.a.nbra * bp.a.nket;
      tk.resize(nq);
      for (int q = 0; q < nq; ++q) tk[q] = make_int2(0, q);
      HIP_TRY(hipMemcpyAsync(dev(o_tasks), tk.data(), sizeof(int2) * nq, hipMemcpyHostToDevice, s));
      float best = 1e30f;
      std::array<int, 3> bestc = bp.cands[0];
      for (auto &cd : bp.cands) {
        one[0] = bp.a;
        one[0].npt = cd[0];
        one[0].nps = cd[1];
        one[0].dbuf = cd[2];
        one[0].Nhb_pad = 16 * cd[0] * cd[1];
        HIP_TRY(hipMemcpyAsync(dev(o_blocks), one.data(), sizeof(Eri4Args), hipMemcpyHostToDevice, s));
        const int waves = one[0].nct * cd[1] + 1;
        const size_t lds = block_lds(one[0]);
        const int grid = group_grid(lds, waves, nq, eri4_tasks_occupancy(cd[0], bp.a.L, waves));
        // the first run warms caches; the best of three after it (a block's
        // tasks alone take tens of microseconds, so one timing is noisy)
        float ms = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          HIP_TRY(hipEventRecord(e0, s));
          HIP_TRY(launch_eri4_tasks((const Eri4Args *)dev(o_blocks), (const int2 *)dev(o_tasks), nq, cd[0], bp.a.L,
                                    waves, lds, grid, s));
          HIP_TRY(hipEventRecord(e1, s));
          HIP_TRY(hipEventSynchronize(e1));
          float t = 0.0f;
          HIP_TRY(hipEventElapsedTime(&t, e0, e1));
          if (rep > 0) ms = std::min(ms, t);
        }
        if (ms < best) {
          best = ms;
          bestc = cd;
        }
      }
      bp.cands = {bestc};
      c->tune[bp.sig] = bestc;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  // groups: blocks sharing (npt, producer bucket)
  std::map<std::pair<int, int>, std::vector<int>> gmap;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    BlockPlan &bp = blocks[bi];
    const std::array<int, 3> cd = bp.cands[0];
    bp.a.npt = cd[0];
    bp.a.nps = cd[1];
    bp.a.dbuf = cd[2];
    bp.a.Nhb_pad = 16 * cd[0] * cd[1];
    gmap[{cd[0], eri4_lm_bucket(bp.a.L)}].push_back((int)bi);
  }
  std::vector<Eri4Args> dblocks(blocks.size());
  std::vector<int2> tasks;
  tasks.reserve(ntask_all);
  size_t bslot = 0;
  for (auto &gkv : gmap) {
    TaskGroup g{};
    g.npt = gkv.first.first;
    g.Lmax = 0;
    g.waves = 2;
    g.lds = 0;
    const size_t first_block = bslot, first_task = tasks.size();
    std::vector<std::pair<double, int2>> tl;
    for (int bi : gkv.second) {
      const BlockPlan &bp = blocks[bi];
      dblocks[bslot] = bp.a;
      eri4_fill_wtask(dblocks[bslot]);
      g.Lmax = std::max(g.Lmax, bp.a.L);
      g.waves = std::max(g.waves, bp.a.nct * bp.a.nps + 1);
      g.lds = std::max(g.lds, block_lds(bp.a));
      const double cost = block_cost(bp);
      const int nq = bp.a.nbra * bp.a.nket;
      for (int q = 0; q < nq; ++q) {
        const int ij = q % bp.a.nbra, kl = q / bp.a.nbra;
        const std::vector<int> &bo = bside[bp.bc].off, &ao = aside[bp.l].off;
        const double w = cost * (bo[ij + 1] - bo[ij]) * (ao[kl + 1] - ao[kl]);
        tl.push_back({w, make_int2((int)(bslot - first_block), q)});
      }
      ++bslot;
    }
    std::stable_sort(tl.begin(), tl.end(), [](const std::pair<double, int2> &x, const std::pair<double, int2> &y) {
      return x.first > y.first;
    });
    for (auto &t : tl) tasks.push_back(t.second);
    g.ntask = (int)tl.size();
    g.d_blocks = (const Eri4Args *)dev(o_blocks) + first_block;
    g.d_tasks = (const int2 *)dev(o_tasks) + first_task;
    g.grid = group_grid(g.lds, g.waves, g.ntask, eri4_tasks_occupancy(g.npt, g.Lmax, g.waves));
    plan->groups.push_back(g);
  }
  HIP_TRY(hipMemcpyAsync(dev(o_blocks), dblocks.data(), sizeof(Eri4Args) * dblocks.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(dev(o_tasks), tasks.data(), sizeof(int2) * tasks.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // host vectors above go out of scope
  // keep at most 8 plans
  if (c->plans.size() >= 8) {
    HIP_TRY(hipDeviceSynchronize());
    free_plan(c->plans.front());
    c->plans.erase(c->plans.begin());
  }
  c->plans.push_back(plan);
  if (flags & MDERI_FLAG_GRAPH) {
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    st = launch_plan(c, plan, c->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    if (st) return st;
    if (ec != hipSuccess) return fail(MDERI_EDEVICE, "mderi_eri3_batch: graph capture failed (%s)", hipGetErrorString(ec));
    plan->graph = graph;
    HIP_TRY(hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0));
    HIP_TRY(hipGraphLaunch(plan->exec, s));
    return MDERI_OK;
  }
  // pair data was already produced on s above; run the groups
  return launch_groups(c, plan, s);
}


// ---------------------------------------------------------------------------
// screened quartet engine: J and K builds and the nuclear gradient (kx.hip)
// ---------------------------------------------------------------------------
namespace {

// One finished launch group of the quartet engine (printed from the stream's
// host-function thread once the group's kernel is done).
struct ProgressMsg {
  int group, ngroup, L, grad;
  long nq;
  std::chrono::steady_clock::time_point t0;
};

void progress_line(void *p) {
  const ProgressMsg *m = (const ProgressMsg *)p;
  const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - m->t0).count();
  fprintf(stderr, "mderi: %s group %d/%d done (total degree %d, %ld quartets) at %.1f s\n",
          m->grad ? "gradient" : "J/K build", m->group + 1, m->ngroup, m->L, m->nq, s);
  fflush(stderr);
  delete m;
}

// What one engine call computes.
struct KxJob {
  bool grad = false;
  // digest mode
  const double *dm = nullptr;
  double *kx = nullptr, *jx = nullptr;
  const double *fscale = nullptr;  // deterministic digest: kx / jx hold fixed-point pairs scaled by *fscale
  // gradient mode
  const double *wl = nullptr, *wr = nullptr;
  int pattern = 0;
  int symmetric = 0;
  double scale = 1.0;
  double *gpart = nullptr;
  int gcopies = 1, gstride = 0;
  int gfixed = 0;  // deterministic: gpart holds four-digit fixed-point words
};

// Per class: its significant pairs (sorted by decreasing Q), sizes, and the
// metadata / pair data of the roles it plays.
struct KxClass {
  int la = 0, lb = 0, Lc = 0, NA = 0, NA_pad = 0, NhB = 0, NhB_pad = 0, maxpp = 0;
  bool asA = false, asB = false;
  bool a6 = false, arel = false;  // gradient A role: in two-visit / one-visit blocks
  int LA = 0, NhA = 0, nh_alloc = 0, LmaxA = 0, S1 = 0, S2 = 0;  // A role (LA includes the +1 of gradients)
  std::vector<double> q;
  std::vector<int32_t> sh;
  size_t o_pp = 0, o_off = 0, o_sh = 0, o_order = 0, o_shift = 0, o_GA = 0, o_HA = 0, o_GB = 0, o_HB = 0;
};

// Largest Y accumulator (doubles) a gradient block keeps in LDS; blocks whose
// A side needs more take the derivative dot products per quartet.
constexpr int kYaccMax = 4608;

// For every row of an A-role order: the rows of (t+1,u,v), (t,u+1,v) and
// (t,u,v+1), 10 bits each (row 0 where the order has no such function).
std::vector<uint32_t> shift_rows(const std::vector<uint32_t> &order) {
  std::map<uint32_t, int> at;
  for (size_t r = 0; r < order.size(); ++r)
    if (!(order[r] & kPadRow) && !at.count(order[r])) at[order[r]] = (int)r;
  std::vector<uint32_t> out(order.size(), 0u);
  for (size_t r = 0; r < order.size(); ++r) {
    if (order[r] & kPadRow) continue;
    const int t = order[r] & 0xff, u = (order[r] >> 8) & 0xff, v = (order[r] >> 16) & 0xff;
    const uint32_t nb[3] = {pack3(t + 1, u, v), pack3(t, u + 1, v), pack3(t, u, v + 1)};
    uint32_t w = 0;
    for (int x = 0; x < 3; ++x) {
      auto it = at.find(nb[x]);
      w |= (uint32_t)(it == at.end() ? 0 : it->second) << (10 * x);
    }
    out[r] = w;
  }
  return out;
}

struct KxPlanBlock {
  int cA, cB, same, onev, yacc, L, npt, nparts, S1, S2;
  long nq;
  double cost;  // rough cycles of one quartet on one wave
  std::vector<long> pre;
  size_t o_pre = 0;
  KxBlock blk{};
};

// One rough cost of a quartet (cycles of one wave): matrix-core steps of the
// two products plus the R build.
double kx_cost(int NhA, int NA, int NhB_pad, int NB, int L, int nct) {
  const int rt = (NhA + 15) / 16, at = (NA + 15) / 16;
  const double mf = (double)nct * rt * (NhB_pad / 4) + (double)nct * at * rt * 4;
  return 64.0 * mf + 40.0 * ntil(L) + 1500.0;
}

mderi_status run_kx(mderi_ctx *c, mderi_basis *b, const PairSets &ps, double tau, const KxJob &job, hipStream_t s) {
  const int ncls = (int)ps.cls.size();
  std::vector<KxClass> C(ncls);
  const int gextra = job.grad ? 1 : 0;
  for (int ci = 0; ci < ncls; ++ci) {
    if (ps.cls[ci].empty()) continue;
    KxClass &k = C[ci];
    const Side &sd = ps.sides[ci];
    k.la = sd.la;
    k.lb = sd.lb;
    k.Lc = k.la + k.lb;
    k.NA = nsph(k.la) * nsph(k.lb);
    k.NA_pad = round16(k.NA);
    k.NhB = ntil(k.Lc);
    k.NhB_pad = (k.NhB + 7) & ~7;
    k.LA = k.Lc + gextra;
    k.NhA = ntil(k.LA);
    for (size_t i = 0; i + 1 < sd.off.size(); ++i) k.maxpp = std::max(k.maxpp, sd.off[i + 1] - sd.off[i]);
    for (int p : ps.cls[ci]) {
      k.q.push_back(ps.q[p]);
      k.sh.push_back(ps.pairs[2 * p]);
      k.sh.push_back(ps.pairs[2 * p + 1]);
    }
  }
  // blocks: unordered class pairs for the builds, and for the gradient
  // when every pair of both classes is a single primitive pair (one visit
  // supplies all four centres); the cheaper orientation.  Otherwise the
  // gradient takes ordered class pairs (each visit supplies its A centres).
  std::vector<KxPlanBlock> blocks;
  for (int x = 0; x < ncls; ++x)
    for (int y = 0; y < ncls; ++y) {
      if (C[x].q.empty() || C[y].q.empty()) continue;
      const bool onev = job.grad && C[x].maxpp == 1 && C[y].maxpp == 1;
      const bool unordered = !job.grad || onev;
      if (unordered && y < x) continue;
      int cA = x, cB = y;
      auto cost_of = [&](int u, int v) {
        const KxClass &A = C[u], &B = C[v];
        return kx_cost(A.NhA, A.NA, B.NhB_pad, B.NA, A.LA + B.Lc, B.NA_pad / 16);
      };
      if (onev) {
        // the A side carries the derivative matrices and the Y accumulator:
        // the lighter pair class takes that role
        const long wx = (long)C[x].NhA * C[x].NA_pad, wy = (long)C[y].NhA * C[y].NA_pad;
        if (wy < wx || (wy == wx && cost_of(y, x) < cost_of(x, y))) std::swap(cA, cB);
      } else if (unordered && x != y && cost_of(y, x) < cost_of(x, y)) {
        std::swap(cA, cB);
      }
      KxPlanBlock pb{};
      pb.cA = cA;
      pb.cB = cB;
      pb.same = (cA == cB) ? 1 : 0;
      pb.onev = onev ? 1 : 0;
      const KxClass &A = C[cA], &B = C[cB];
      pb.L = A.LA + B.Lc;
      const int nA = (int)A.q.size();
      pb.pre.assign(nA + 1, 0);
      for (int i = 0; i < nA; ++i) {
        // B pairs k with Q_i Q_k >= tau: a prefix of the sorted list
        int lo = 0, hi = (int)B.q.size();
        while (lo < hi) {
          const int mid = (lo + hi) / 2;
          if (A.q[i] * B.q[mid] >= tau) lo = mid + 1;
          else hi = mid;
        }
        long cnt = lo;
        if (pb.same && unordered) cnt = std::min<long>(cnt, i + 1);
        pb.pre[i + 1] = pb.pre[i] + cnt;
      }
      pb.nq = pb.pre[nA];
      if (pb.nq == 0) continue;
      const int ntiles = (A.NhA + 15) / 16;
      // gradient kernels hold more state per wave: at most two row tiles
      pb.npt = ntiles <= 1 ? 1 : (ntiles <= 2 || job.grad) ? 2 : 4;
      pb.nparts = (ntiles + pb.npt - 1) / pb.npt;
      pb.cost = kx_cost(A.NhA, A.NA, B.NhB_pad, B.NA, pb.L, B.NA_pad / 16);
      if (pb.L > 18) return fail(MDERI_EUNSUPPORTED, "quartet class of total degree %d is beyond the engine", pb.L);
      blocks.push_back(std::move(pb));
      C[cA].asA = true;
      if (job.grad) (onev ? C[cA].arel : C[cA].a6) = true;
      C[cB].asB = true;
      C[cA].nh_alloc = std::max(C[cA].nh_alloc, blocks.back().nparts * blocks.back().npt * 16);
      C[cA].LmaxA = std::max(C[cA].LmaxA, blocks.back().L);
    }
  if (blocks.empty()) return MDERI_OK;
  // A-role row order: bank-spread for the strides of the class's largest block
  for (auto &k : C)
    if (k.asA) choose_cube(k.LmaxA, k.LA, &k.S1, &k.S2);
  for (auto &pb : blocks) choose_cube(pb.L, C[pb.cA].LA, &pb.S1, &pb.S2);

  // launch groups by (row tiles, total degree, size of the gradient's
  // accumulator and staging): the wave's LDS regions are sized for its
  // group, so blocks with small regions keep their occupancy; heaviest
  // quartets first inside a group
  std::map<std::array<int, 3>, std::vector<int>> groups;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    const KxPlanBlock &pb = blocks[bi];
    const KxClass &A = C[pb.cA];
    int extra = 0;
    if (job.grad) {
      const int rows = std::max(A.nh_alloc, round16(A.NhA)), y = A.maxpp * rows * A.NA_pad;
      extra = (y <= kYaccMax ? y : 0) + (pb.onev ? 17 * rows : 0);
    }
    const int bucket = extra <= 1024 ? 0 : extra <= 2048 ? 1 : extra <= 3072 ? 2 : 3;
    groups[{pb.npt, pb.L, bucket}].push_back((int)bi);
  }
  for (auto &gr : groups)
    std::stable_sort(gr.second.begin(), gr.second.end(),
                     [&](int x, int y) { return blocks[x].cost > blocks[y].cost; });

  // metadata image: per class pairs, offsets, shells, A order; per block pre;
  // per group the block descriptors; then the device-only pair data
  Image img;
  for (int ci = 0; ci < ncls; ++ci) {
    KxClass &k = C[ci];
    if (!k.asA && !k.asB) continue;
    const Side &sd = ps.sides[ci];
    k.o_pp = img.add(sd.pp.data(), sizeof(PrimPair) * sd.pp.size());
    k.o_off = img.add(sd.off.data(), sizeof(int) * sd.off.size());
    k.o_sh = img.add(k.sh.data(), sizeof(int32_t) * k.sh.size());
    if (k.asA) {
      std::vector<uint32_t> order = bra_row_order(k.LA, k.S1, k.S2, round16(k.NhA));
      while ((int)order.size() < k.nh_alloc) order.push_back(order[0] | kPadRow);
      order.resize(std::max<size_t>(order.size(), (size_t)k.nh_alloc));
      k.nh_alloc = (int)order.size();
      k.o_order = img.add(order.data(), sizeof(uint32_t) * order.size());
      if (k.nh_alloc > 1024) return fail(MDERI_EUNSUPPORTED, "quartet engine: %d A rows", k.nh_alloc);
      const std::vector<uint32_t> sh = shift_rows(order);
      k.o_shift = img.add(sh.data(), sizeof(uint32_t) * sh.size());
    }
  }
  for (auto &pb : blocks) pb.o_pre = img.add(pb.pre.data(), sizeof(long) * pb.pre.size());
  struct Group {
    int npt, lm, waves, grid;
    size_t lds;
    long nchunk;
    KxArgs args;
    size_t o_blocks, o_counter;
    std::vector<KxBlock> blks;
  };
  std::vector<Group> G;
  for (auto &gr : groups) {
    Group g{};
    g.npt = gr.first[0];
    g.lm = gr.first[1];  // total degree L: the producer bucket follows it
    g.blks.resize(gr.second.size());
    g.o_blocks = img.add(g.blks.data(), sizeof(KxBlock) * g.blks.size());  // filled in below
    G.push_back(std::move(g));
  }
  const size_t meta_bytes = img.bytes.size();
  // matrices per primitive pair: A role 7 in gradient mode (six derivative
  // matrices and the plain one), B role 4 for single-primitive classes in
  // gradient mode (plain and three relative-coordinate derivatives)
  // A role in gradient mode: six derivative matrices (two-visit blocks), the
  // plain matrix, three d/d(A-B) matrices (one-visit blocks)
  auto matsA = [&](const KxClass &k) { return (k.a6 ? 6 : 0) + 1 + (k.arel ? 3 : 0); };
  auto matsB = [&](const KxClass &k) { return (job.grad && k.maxpp == 1) ? 4 : 1; };
  for (auto &k : C) {
    const int npp = (int)ps.sides[&k - &C[0]].pp.size();
    if (k.asA) {
      k.o_GA = img.add(nullptr, sizeof(double) * 4 * npp);
      k.o_HA = img.add(nullptr, sizeof(double) * matsA(k) * (size_t)k.nh_alloc * k.NA_pad * npp);
    }
    if (k.asB) {
      k.o_GB = img.add(nullptr, sizeof(double) * 4 * npp);
      k.o_HB = img.add(nullptr, sizeof(double) * matsB(k) * (size_t)k.NhB_pad * k.NA_pad * npp);
    }
  }
  for (auto &g : G) g.o_counter = img.add(nullptr, sizeof(unsigned long long));
  mderi_status st;
  void *dmem;
  if ((st = ws_get(c, WS_PAIRS, img.size, &dmem))) return st;
  char *base = (char *)dmem;
  auto dev = [&](size_t off) { return (void *)(base + off); };

  // block descriptors, chunks and per-wave LDS layout of every group
  size_t gi = 0;
  for (auto &gr : groups) {
    Group &g = G[gi++];
    int cube_max = 2, work_max = 2, v_max = 2, d_max = 2, i_max = 2, g_max = 4, uv_max = 1, oq_max = 8, op_max = 16;
    int y_max = 0, x_max = 0;
    bool single = true;  // every quartet is one primitive quartet: v may share the work area
    double work = 0.0;  // estimated cycles of the whole group
    for (size_t j = 0; j < gr.second.size(); ++j) {
      KxPlanBlock &pb = blocks[gr.second[j]];
      const KxClass &A = C[pb.cA], &B = C[pb.cB];
      KxBlock &x = g.blks[j];
      x.nq = pb.nq;
      work += (double)pb.nq * pb.cost;
      x.pre = (const long *)dev(pb.o_pre);
      x.nA = (int)A.q.size();
      x.L = pb.L;
      x.S1 = pb.S1;
      x.S2 = pb.S2;
      x.NhA = A.NhA;
      x.HA_rows = A.nh_alloc;
      x.nparts = pb.nparts;
      x.NhB = B.NhB;
      x.NhB_pad = B.NhB_pad;
      x.NA = A.NA;
      x.NB = B.NA;
      x.NA_pad = A.NA_pad;
      x.NB_pad = B.NA_pad;
      x.nct = B.NA_pad / 16;
      x.na = nsph(A.la);
      x.nb = nsph(A.lb);
      x.nc = nsph(B.la);
      x.nd = nsph(B.lb);
      x.same = pb.same;
      x.onev = pb.onev;
      x.yacc = job.grad && A.maxpp * A.nh_alloc * A.NA_pad <= kYaccMax ? 1 : 0;
      x.Ashift = (const uint32_t *)dev(A.o_shift);
      x.A_mats = matsA(A);
      x.A_plain = A.a6 ? 6 : 0;
      x.A_rel = x.A_plain + 1;
      x.A_pp = (const PrimPair *)dev(A.o_pp);
      x.B_mats = matsB(B);
      x.B_pp = (const PrimPair *)dev(B.o_pp);
      x.inv_nb = 1.0f / (float)x.nb;
      x.inv_nd = 1.0f / (float)x.nd;
      x.inv_NB = 1.0f / (float)x.NB;
      x.inv_ncd = 1.0f / (float)(x.nc + x.nd);
      x.Aorder = (const uint32_t *)dev(A.o_order);
      x.A_off = (const int *)dev(A.o_off);
      x.B_off = (const int *)dev(B.o_off);
      x.A_G = (const double *)dev(A.o_GA);
      x.A_H = (const double *)dev(A.o_HA);
      x.B_G = (const double *)dev(B.o_GB);
      x.B_H = (const double *)dev(B.o_HB);
      x.A_sh = (const int *)dev(A.o_sh);
      x.B_sh = (const int *)dev(B.o_sh);
      const int nab = x.na + x.nb, ncd = x.nc + x.nd;
      cube_max = std::max(cube_max, (pb.L * pb.S1 + 2) & ~1);
      work_max = std::max(work_max, rr_work_size(pb.L));
      v_max = std::max(v_max, x.NA_pad * 16);  // one B column tile of V or of the weights
      int d = 0, im = 0;
      if (job.grad) d = job.pattern == 0 ? (job.symmetric ? 1 : 4) * nab * ncd : 2 * (x.NA + x.NB);
      else d = im = (job.kx ? nab * ncd : 0) + (job.jx ? x.NA + x.NB : 0);
      d_max = std::max(d_max, d);
      i_max = std::max(i_max, im);
      single = single && A.maxpp == 1 && B.maxpp == 1;
      g_max = std::max(g_max, 4 * (A.maxpp + B.maxpp));
      uv_max = std::max(uv_max, (pb.L + 1) * (pb.L + 2) / 2);
      if (x.yacc) y_max = std::max(y_max, A.maxpp * A.nh_alloc * A.NA_pad);
      if (x.onev) x_max = std::max(x_max, 17 * A.nh_alloc);
      oq_max = std::max(oq_max, round16(x.NhB_pad));
      op_max = std::max(op_max, x.HA_rows);
    }
    auto even = [](int v) { return (v + 1) & ~1; };
    KxArgs &ar = g.args;
    ar.o_work = even(cube_max);
    ar.o_v = single ? ar.o_work : ar.o_work + even(work_max);
    ar.o_d = single ? ar.o_work + even(std::max(work_max, v_max)) : ar.o_v + even(v_max);
    ar.o_img = ar.o_d + even(d_max);
    ar.o_g = ar.o_img + even(i_max);
    ar.o_y = ar.o_g + even(g_max);
    ar.o_x = ar.o_y + even(y_max);
    ar.o_tab = ar.o_x + even(x_max);
    ar.uv_max = even(uv_max);
    ar.oq_max = even(oq_max);
    ar.op_max = even(op_max);
    ar.wave_doubles = ar.o_tab + (ar.uv_max + ar.oq_max + 2 * ar.op_max + 1) / 2 + 1;
    ar.wave_doubles = even(ar.wave_doubles);
    const size_t wave_bytes = sizeof(double) * (size_t)ar.wave_doubles;
    if (wave_bytes > 160 * 1024)
      return fail(MDERI_EUNSUPPORTED, "quartet engine: a wave needs %zu bytes of LDS (over 160 KiB)", wave_bytes);
    // waves are independent (each has its own LDS region and takes its own
    // chunks), so the workgroup size only decides how many waves the CU's
    // LDS holds: 4 per workgroup leaves up to 3 waves' worth unused.  Take
    // the size that holds the most waves, counting at most the waves the
    // registers allow (the digest's 72-104 VGPRs: 32 per CU are counted, as
    // the grid always did; the gradient's up to 256: 8), ties going to the
    // larger workgroup.
    const size_t wave_cap = job.grad ? 8 : 32;
    g.waves = 1;
    size_t best = 0;
    for (int w = 4; w >= 1; --w) {
      const size_t tot = std::min<size_t>(wave_cap, w * ((160 * 1024) / (wave_bytes * w)));
      if (tot > best) {
        best = tot;
        g.waves = w;
      }
    }
    g.lds = wave_bytes * g.waves;
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(wave_cap / g.waves, (160 * 1024) / g.lds));
    // chunks: at least ~7.5e4 cycles each (the per-chunk search and table
    // set-up stay small), and larger where the group's work allows about
    // 128 chunks per resident wave (measured on the 40-atom cluster: 16
    // and 32 per wave were 1-3% slower for the K build and the gradient);
    // blocks run heaviest first, so the tail is made of the cheapest
    // block's chunks
    const double per_chunk = std::max(7.5e4, work / (128.0 * 256.0 * per_cu * g.waves));
    long chunk0 = 0;
    for (size_t j = 0; j < gr.second.size(); ++j) {
      const KxPlanBlock &pb = blocks[gr.second[j]];
      KxBlock &x = g.blks[j];
      x.chunk = (int)std::max(1.0, std::min(4096.0, per_chunk / pb.cost));
      x.chunk0 = chunk0;
      chunk0 += (pb.nq + x.chunk - 1) / x.chunk;
    }
    g.nchunk = chunk0;
    g.grid = (int)std::min<long>(256L * per_cu, std::max<long>(1, (g.nchunk + g.waves - 1) / g.waves));
    ar.blocks = (const KxBlock *)dev(g.o_blocks);
    ar.nblk = (int)g.blks.size();
    ar.nchunk = g.nchunk;
    ar.counter = (unsigned long long *)dev(g.o_counter);
    ar.tab = c->tab;
    ar.ao_off = b->dev.ao_off;
    ar.nao = b->nao;
    ar.dm = job.dm;
    ar.kx = job.kx;
    ar.jx = job.jx;
    ar.fixed = job.fscale ? 1 : 0;
    ar.fscale = job.fscale;
    ar.wl = job.wl;
    ar.wr = job.wr;
    ar.pattern = job.pattern;
    ar.symmetric = job.symmetric;
    ar.scale = job.scale;
    ar.grad = job.gpart;
    ar.gcopies = job.gcopies;
    ar.gstride = job.gstride;
    ar.gfixed = job.gfixed;
    ar.atom = b->dev.atom;
    ar.exps = b->dev.exps;
    memcpy(img.bytes.data() + g.o_blocks, g.blks.data(), sizeof(KxBlock) * g.blks.size());
  }

  if ((st = stage_begin(c, meta_bytes))) return st;
  size_t used = 0;
  if ((st = stage_copy(c, base, img.bytes.data(), meta_bytes, s, &used))) return st;
  if ((st = stage_end(c, s))) return st;
  // pair data once per class and role
  for (int ci = 0; ci < ncls; ++ci) {
    const KxClass &k = C[ci];
    if (!k.asA && !k.asB) continue;
    const Side &sd = ps.sides[ci];
    PairArgs pa{};
    pa.basis = b->dev;
    pa.tab = c->tab;
    pa.npp = (int)sd.pp.size();
    pa.pp = (const PrimPair *)dev(k.o_pp);
    pa.la = k.la;
    pa.lb = k.lb;
    pa.N = k.NA;
    pa.N_pad = k.NA_pad;
    if (k.asA) {
      pa.Nh = k.NhA;
      pa.Nh_pad = k.nh_alloc;
      pa.deriv = k.a6 ? 1 : 0;
      pa.rderiv = k.arel ? 1 : 0;
      pa.rtrans = 1;
      pa.order = (const uint32_t *)dev(k.o_order);
      pa.ket_sign = 0;
      pa.G = (double *)dev(k.o_GA);
      pa.H = (double *)dev(k.o_HA);
      HIP_TRY(launch_pairs(pa, s));
    }
    if (k.asB) {
      pa.Nh = k.NhB;
      pa.Nh_pad = k.NhB_pad;
      pa.deriv = 0;
      pa.rderiv = matsB(k) == 4 ? 1 : 0;
      pa.rtrans = 0;
      pa.order = nullptr;
      pa.ket_sign = 1;
      pa.G = (double *)dev(k.o_GB);
      pa.H = (double *)dev(k.o_HB);
      HIP_TRY(launch_pairs(pa, s));
    }
  }
  const auto t_start = std::chrono::steady_clock::now();
  for (auto &g : G) {
    HIP_TRY(launch_zero(1, (double *)dev(g.o_counter), s));  // chunk counter (zero bits)
    if (c->timing) {
      if (c->ev_free.empty()) {
        std::pair<hipEvent_t, hipEvent_t> e;
        HIP_TRY(hipEventCreate(&e.first));
        HIP_TRY(hipEventCreate(&e.second));
        c->ev_free.push_back(e);
      }
      const auto e = c->ev_free.back();
      c->ev_free.pop_back();
      c->ev_used.push_back(e);
      HIP_TRY(hipEventRecord(e.first, s));
      HIP_TRY(launch_kx(g.args, g.npt, g.lm, job.grad, g.waves, g.lds, g.grid, s));
      HIP_TRY(hipEventRecord(e.second, s));
    } else {
      HIP_TRY(launch_kx(g.args, g.npt, g.lm, job.grad, g.waves, g.lds, g.grid, s));
    }
    if (c->progress) {
      long nq = 0;
      for (const KxBlock &x : g.blks) nq += x.nq;
      ProgressMsg *m = new ProgressMsg{(int)(&g - &G[0]), (int)G.size(), g.lm, job.grad ? 1 : 0, nq, t_start};
      const hipError_t e = hipLaunchHostFunc(s, progress_line, m);
      if (e != hipSuccess) {
        delete m;
        HIP_TRY(e);
      }
    }
  }
  return MDERI_OK;
}

double opt_tau(const mderi_opts *opts) { return (opts && opts->schwarz_tau > 0.0) ? opts->schwarz_tau : 1e-12; }

}  // namespace

extern "C" mderi_status mderi_jkbuild(mderi_ctx_t c, mderi_basis_t b, const double *D, double *J, double *K, int nao,
                                      double *energy, const mderi_opts *opts, void *stream) {
  mderi_status st;
  if ((st = check_density("mderi_jkbuild", c, b, D, nao, opts))) return st;
  if (!J && !K) return fail(MDERI_EINVAL, "mderi_jkbuild: J and K are both NULL");
  const double tau = opt_tau(opts);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  std::shared_ptr<const PairSets> psel;
  if ((st = select_pairs(c, b, tau, s, psel))) return st;
  const PairSets &ps = *psel;
  const size_t nn = (size_t)nao * nao;
  // deterministic: 2 64-bit words per element and the scale; else one double
  const bool det = opts && opts->deterministic;
  const size_t per = det ? 2 * nn : nn, nmat = (J ? 1 : 0) + (K ? 1 : 0);
  const size_t nwork = std::max(dot2_work_doubles(), det_scale_work_doubles()) + 1;
  void *d_t;
  if ((st = ws_get(c, WS_KTMP, sizeof(double) * (per * nmat + nwork), &d_t))) return st;
  double *kt = K ? (double *)d_t : nullptr;
  double *jt = J ? (double *)d_t + (K ? per : 0) : nullptr;
  double *work = (double *)d_t + per * nmat;
  double *scale = work + nwork - 1;
  if (kt) HIP_TRY(det ? launch_zero_u64(per, (unsigned long long *)kt, s) : launch_zero(nn, kt, s));
  if (jt) HIP_TRY(det ? launch_zero_u64(per, (unsigned long long *)jt, s) : launch_zero(nn, jt, s));
  if (det) {
    double qmax = 0.0;
    for (double q : ps.q) qmax = std::max(qmax, q);
    HIP_TRY(launch_det_scale(nn, D, qmax, work, scale, s));
  }
  KxJob job;
  job.dm = D;
  job.kx = kt;
  job.jx = jt;
  job.fscale = det ? scale : nullptr;
  if ((st = run_kx(c, b, ps, tau, job, s))) return st;
  if (det) {
    if (K) HIP_TRY(launch_symmetrize_fixed(nao, (const unsigned long long *)kt, scale, K, s));
    if (J) HIP_TRY(launch_symmetrize_fixed(nao, (const unsigned long long *)jt, scale, J, s));
  } else {
    if (K) HIP_TRY(launch_symmetrize(nao, kt, K, s));
    if (J) HIP_TRY(launch_symmetrize(nao, jt, J, s));
  }
  if (energy) HIP_TRY(launch_dot2(nn, D, J, K, work, energy, s));
  return MDERI_OK;
}

extern "C" mderi_status mderi_kbuild(mderi_ctx_t c, mderi_basis_t b, const double *D, double *K, int nao,
                                     const mderi_opts *opts, void *stream) {
  if (!K) return fail(MDERI_EINVAL, "mderi_kbuild: NULL output");
  return mderi_jkbuild(c, b, D, nullptr, K, nao, nullptr, opts, stream);
}

extern "C" mderi_status mderi_basis_set_centers(mderi_basis_t b, const double *centers, void *stream) {
  if (!b) return fail(MDERI_EINVAL, "mderi_basis_set_centers: NULL basis");
  if (!centers) return fail(MDERI_EINVAL, "mderi_basis_set_centers: NULL centres");
  HIP_TRY(hipSetDevice(b->ctx->device));
  // the cached pair selections of the old geometry no longer hold
  ++b->geom;
  drop_pair_selections(b);
  HIP_TRY(hipMemcpyAsync(b->dev.centers, centers, sizeof(double) * 3 * (size_t)b->nshell, hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return MDERI_OK;
}

extern "C" mderi_status mderi_kbuild_grad(mderi_ctx_t c, mderi_basis_t b, int pattern, const double *Wl,
                                          const double *Wr, int nao, double scale, double *grad, int natom,
                                          int accumulate, const mderi_opts *opts, void *stream) {
  mderi_status st;
  if ((st = check_density("mderi_kbuild_grad", c, b, Wl, nao, opts))) return st;
  if (!Wr) return fail(MDERI_EINVAL, "mderi_kbuild_grad: NULL Wr");
  if (pattern != MDERI_EXCHANGE && pattern != MDERI_COULOMB)
    return fail(MDERI_EINVAL, "mderi_kbuild_grad: pattern %d", pattern);
  if (!grad) return fail(MDERI_EINVAL, "mderi_kbuild_grad: NULL output");
  if (natom <= 0) return fail(MDERI_EINVAL, "mderi_kbuild_grad: natom %d", natom);
  if (!std::isfinite(scale)) return fail(MDERI_EINVAL, "mderi_kbuild_grad: scale is not finite");
  for (int i = 0; i < b->nshell; ++i)
    if (b->atom[i] < 0 || b->atom[i] >= natom)
      return fail(MDERI_EINVAL, "mderi_kbuild_grad: shell %d sits on atom %d, outside [0,%d)", i, b->atom[i], natom);
  const double tau = opt_tau(opts);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  std::shared_ptr<const PairSets> psel;
  if ((st = select_pairs(c, b, tau, s, psel))) return st;
  const PairSets &ps = *psel;
  // the waves add into kGradCopies partial gradients (by workgroup), summed
  // into grad at the end, so the atomics of many short flushes do not queue
  // on the same 3 natom addresses
  constexpr int kGradCopies = 512;
  // deterministic: four 64-bit digit words per element instead of one double
  const bool det = opts && opts->deterministic;
  const size_t nwords = (size_t)kGradCopies * 3 * natom * (det ? 4 : 1);
  void *d_gpart = nullptr;
  if ((st = ws_get(c, WS_GPART, sizeof(double) * nwords, &d_gpart))) return st;
  HIP_TRY(det ? launch_zero_u64(nwords, (unsigned long long *)d_gpart, s) : launch_zero(nwords, (double *)d_gpart, s));
  KxJob job;
  job.grad = true;
  job.wl = Wl;
  job.wr = Wr;
  job.pattern = pattern;
  job.symmetric = ((opts ? opts->flags : 0) & MDERI_FLAG_SYMMETRIC) && Wl == Wr ? 1 : 0;
  job.scale = scale;
  job.gpart = (double *)d_gpart;
  job.gcopies = kGradCopies;
  job.gstride = 3 * natom;
  job.gfixed = det ? 1 : 0;
  if ((st = run_kx(c, b, ps, tau, job, s))) return st;
  if (det)
    HIP_TRY(launch_sum_copies_fixed(3 * natom, kGradCopies, (const unsigned long long *)d_gpart, grad,
                                    accumulate ? 1 : 0, s));
  else
    HIP_TRY(launch_sum_copies(3 * natom, kGradCopies, (const double *)d_gpart, grad, s, accumulate ? 1 : 0));
  return MDERI_OK;
}

// ---------------------------------------------------------------------------
// density-fitted Coulomb matrix
// ---------------------------------------------------------------------------
namespace {

// The shared part of the density-fitted builds: the (ab|P) matrix B over the
// canonical shell pairs (rows = AO pairs, w = 2 for pairs of two shells, 1 on
// a diagonal shell pair) and every auxiliary AO (columns), the metric M =
// (P|Q) from its class batches, and M's Cholesky factor L (lower, in place of
// M), all enqueued on s.
struct DfSetup {
  int nrow = 0, ncol = 0;
  double *B = nullptr, *M = nullptr, *vec = nullptr;  // vec: nrow + ncol doubles of work
  const int2 *ab = nullptr;
  const double *w = nullptr;
};

// The factors of the fit for (b, aux): taken from the context when its last
// density-fitting call had the same bases at the same geometries (df_stage
// says how far they were carried), else computed (df_stage 1).
mderi_status df_setup(mderi_ctx *c, mderi_basis *b, mderi_basis *aux, const char *fn, hipStream_t s, DfSetup &df) {
  const uint64_t key[4] = {b->serial, b->geom, aux->serial, aux->geom};
  if (c->df_stage && std::equal(key, key + 4, c->df_key)) {
    if (rocblas_set_stream(c->blas, s) != rocblas_status_success)
      return fail(MDERI_EDEVICE, "%s: rocblas_set_stream failed", fn);
    df.nrow = c->df_nrow;
    df.ncol = aux->nao;
    df.B = (double *)c->ws[WS_DFB];
    df.M = (double *)c->ws[WS_DFM];
    df.vec = (double *)c->ws[WS_DFV];
    df.ab = (const int2 *)c->ws[WS_DFI];
    df.w = (const double *)((char *)c->ws[WS_DFI] + sizeof(int2) * (size_t)df.nrow);
    return MDERI_OK;
  }
  c->df_stage = 0;
  std::vector<int32_t> pairs;
  std::vector<int2> ab;
  std::vector<double> w;
  for (int i = 0; i < b->nshell; ++i)
    for (int j = 0; j <= i; ++j) {
      pairs.push_back(i);
      pairs.push_back(j);
      const int Na = nsph(b->l[i]), Nb = nsph(b->l[j]);
      for (int ma = 0; ma < Na; ++ma)
        for (int mb = 0; mb < Nb; ++mb) {
          ab.push_back(make_int2(b->ao_off[i] + ma, b->ao_off[j] + mb));
          w.push_back(i == j ? 1.0 : 2.0);
        }
    }
  const int nrow = (int)ab.size(), ncol = aux->nao, npair = (int)pairs.size() / 2;
  std::vector<int32_t> auxidx(aux->nshell);
  std::iota(auxidx.begin(), auxidx.end(), 0);
  // auxiliary shells ordered by l: the class batches of the metric
  std::vector<int32_t> byl;
  std::vector<int> lstart(kLmax + 2, 0);
  for (int l = 0; l <= kLmax; ++l) {
    for (int k = 0; k < aux->nshell; ++k)
      if (aux->l[k] == l) byl.push_back(k);
    lstart[l + 1] = (int)byl.size();
  }
  size_t maxT = 1;
  for (int la = 0; la <= kLmax; ++la)
    for (int lc = 0; lc <= kLmax; ++lc)
      maxT = std::max(maxT, (size_t)(lstart[la + 1] - lstart[la]) * nsph(la) * nsph(lc) * (lstart[lc + 1] - lstart[lc]));
  mderi_status st;
  void *dB, *dM, *dT, *dV, *dI;
  const size_t o_w = sizeof(int2) * (size_t)nrow, o_byl = o_w + sizeof(double) * (size_t)nrow;
  const size_t ibytes = o_byl + sizeof(int32_t) * byl.size();
  if ((st = ws_get(c, WS_DFB, sizeof(double) * (size_t)nrow * ncol, &dB)) ||
      (st = ws_get(c, WS_DFM, sizeof(double) * (size_t)ncol * ncol, &dM)) ||
      (st = ws_get(c, WS_DFT, sizeof(double) * maxT, &dT)) ||
      (st = ws_get(c, WS_DFV, sizeof(double) * ((size_t)nrow + ncol) + 64, &dV)) ||
      (st = ws_get(c, WS_DFI, ibytes, &dI)))
    return st;
  df.nrow = nrow;
  df.ncol = ncol;
  df.B = (double *)dB;
  df.M = (double *)dM;
  df.vec = (double *)dV;
  df.ab = (const int2 *)dI;
  df.w = (const double *)((char *)dI + o_w);
  const int32_t *d_byl = (const int32_t *)((char *)dI + o_byl);
  if ((st = stage_begin(c, ibytes))) return st;
  size_t used = 0;
  if ((st = stage_copy(c, dI, ab.data(), sizeof(int2) * ab.size(), s, &used)) ||
      (st = stage_copy(c, (char *)dI + o_w, w.data(), sizeof(double) * w.size(), s, &used)) ||
      (st = stage_copy(c, (char *)dI + o_byl, byl.data(), sizeof(int32_t) * byl.size(), s, &used)))
    return st;
  if ((st = stage_end(c, s))) return st;
  // (ab|P) for every canonical pair and auxiliary shell
  mderi_opts o{};
  if ((st = mderi_eri3_batch(c, b, aux, npair, pairs.data(), aux->nshell, auxidx.data(), df.B, (size_t)nrow * ncol,
                             &o, s)))
    return st;
  // the metric (P|Q), class batch by class batch, scattered into M
  for (int la = 0; la <= kLmax; ++la)
    for (int lc = 0; lc <= kLmax; ++lc) {
      const int na = lstart[la + 1] - lstart[la], nc = lstart[lc + 1] - lstart[lc];
      if (!na || !nc) continue;
      Side sa{aux, 0, 0, true, {}, {}}, sc{aux, 0, 0, true, {}, {}};
      if ((st = expand_shells(aux, na, byl.data() + lstart[la], "aux", &sa.la, sa)) ||
          (st = expand_shells(aux, nc, byl.data() + lstart[lc], "aux", &sc.la, sc)))
        return st;
      if ((st = run_class_batch(c, sa, sc, 0, (double *)dT, nullptr, nullptr, s))) return st;
      HIP_TRY(launch_df_scatter(na, nsph(la), nc, nsph(lc), (const double *)dT, d_byl + lstart[la],
                                d_byl + lstart[lc], aux->dev.ao_off, df.M, ncol, s));
    }
  // Cholesky factor of the metric, in place
  if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success)
    return fail(MDERI_EDEVICE, "%s: rocblas_create_handle failed", fn);
  rocblas_int *info = (rocblas_int *)(df.vec + nrow + ncol);
  if (rocblas_set_stream(c->blas, s) != rocblas_status_success ||
      rocsolver_dpotrf(c->blas, rocblas_fill_lower, ncol, df.M, ncol, info) != rocblas_status_success)
    return fail(MDERI_EDEVICE, "%s: the metric factorisation could not be enqueued", fn);
  std::copy(key, key + 4, c->df_key);
  c->df_nrow = nrow;
  c->df_stage = 1;
  return MDERI_OK;
}

mderi_status df_check(mderi_ctx *c, mderi_basis *b, mderi_basis *aux, const double *D, const double *out, int nao,
                      const mderi_opts *opts, const char *fn) {
  if (!c || !b || !aux) return fail(MDERI_EINVAL, "%s: NULL context or basis", fn);
  if (b->ctx != c || aux->ctx != c) return fail(MDERI_EINVAL, "%s: basis belongs to another context", fn);
  if (!D || !out) return fail(MDERI_EINVAL, "%s: NULL density or output", fn);
  if (nao != b->nao) return fail(MDERI_EINVAL, "%s: nao %d but the basis has %d AOs", fn, nao, b->nao);
  if (opts && opts->precision != 0) return fail(MDERI_EUNSUPPORTED, "%s: precision %d", fn, opts->precision);
  return MDERI_OK;
}

}  // namespace

extern "C" mderi_status mderi_dfj(mderi_ctx_t c, mderi_basis_t b, mderi_basis_t aux, const double *D, double *J,
                                  int nao, const mderi_opts *opts, void *stream) {
  mderi_status st;
  if ((st = df_check(c, b, aux, D, J, nao, opts, "mderi_dfj"))) return st;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  DfSetup df;
  if ((st = df_setup(c, b, aux, "mderi_dfj", s, df))) return st;
  // fitted charge gamma_Q = sum w (Q|ab) D_ab, c = M^{-1} gamma, J; when a
  // K build left B' = B L^-T in place of B, gamma' = B'^T d = L^-1 gamma
  // and J = B' gamma' = B M^-1 gamma with no solve
  double *dvec = df.vec, *gamma = dvec + df.nrow;
  HIP_TRY(launch_df_dvec(df.nrow, df.ab, df.w, D, nao, dvec, s));
  HIP_TRY(launch_df_gamma(df.nrow, df.ncol, df.B, dvec, gamma, s));
  if (c->df_stage < 2 && rocsolver_dpotrs(c->blas, rocblas_fill_lower, df.ncol, 1, df.M, df.ncol, gamma,
                                          df.ncol) != rocblas_status_success)
    return fail(MDERI_EDEVICE, "mderi_dfj: the metric solve could not be enqueued");
  HIP_TRY(launch_df_j(df.nrow, df.ncol, df.B, gamma, df.ab, J, nao, s));
  return MDERI_OK;
}

extern "C" mderi_status mderi_dfk(mderi_ctx_t c, mderi_basis_t b, mderi_basis_t aux, const double *D, double *K,
                                  int nao, const mderi_opts *opts, void *stream) {
  mderi_status st;
  if ((st = df_check(c, b, aux, D, K, nao, opts, "mderi_dfk"))) return st;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  const size_t naux = (size_t)aux->nao, n3 = (size_t)nao * nao * naux;
  if (naux * nao > 0x7fffffffu)
    return fail(MDERI_EUNSUPPORTED, "mderi_dfk: %zu x %d exceeds a GEMM dimension", naux, nao);
  DfSetup df;
  if ((st = df_setup(c, b, aux, "mderi_dfk", s, df))) return st;
  void *dBt, *dX, *dK;
  if ((st = ws_get(c, WS_DFK1, sizeof(double) * n3, &dBt)) || (st = ws_get(c, WS_DFK2, sizeof(double) * n3, &dX)) ||
      (st = ws_get(c, WS_DFK3, sizeof(double) * (size_t)nao * nao, &dK)))
    return st;
  double *Bt = (double *)dBt, *X = (double *)dX, *Kt = (double *)dK;
  const double one = 1.0, half = 0.5, zero = 0.0;
  const rocblas_int m = nao, k2 = (rocblas_int)(naux * nao);
  // B' = B L^{-T}: the fitted integrals are (ab|cd)_fit = sum_Q B'[ab][Q] B'[cd][Q]
  if (c->df_stage < 2) {
    if (rocblas_dtrsm(c->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                      rocblas_diagonal_non_unit, df.nrow, df.ncol, &one, df.M, df.ncol, df.B, df.nrow) !=
        rocblas_status_success) {
      c->df_stage = 0;  // B may be half transformed
      return fail(MDERI_EDEVICE, "mderi_dfk: the triangular solve could not be enqueued");
    }
    c->df_stage = 2;
  }
  // Bt[(a naux + Q) nao + b] = B'_Q[a][b] over all AO pairs, then
  // X[(a naux + Q) nao + d] = sum_b D[d][b] B'_Q[a][b]  (one GEMM, k = nao)
  // K~[c + nao a] = 1/2 sum_{Q,d} B'_Q[c][d] X_Q[a][d]  (one GEMM, k = naux nao)
  // and K = K~ + K~^T = sum_Q B'_Q D B'_Q^T, exactly symmetric
  if (c->df_stage < 3) {
    HIP_TRY(launch_df_expand(df.nrow, df.ncol, df.B, df.ab, df.w, nao, Bt, s));
    c->df_stage = 3;
  }
  if (rocblas_dgemm(c->blas, rocblas_operation_none, rocblas_operation_none, m, k2, m, &one, D, m, Bt, m, &zero, X,
                    m) != rocblas_status_success ||
      rocblas_dgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, m, m, k2, &half, Bt, k2, X, k2,
                    &zero, Kt, m) != rocblas_status_success)
    return fail(MDERI_EDEVICE, "mderi_dfk: the contractions could not be enqueued");
  HIP_TRY(launch_symmetrize(nao, Kt, K, s));
  return MDERI_OK;
}

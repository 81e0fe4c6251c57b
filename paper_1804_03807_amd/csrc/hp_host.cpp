// Host side of libhomotopy: argument checking, system packing, device
// buffers, kernel-variant choice (autotuned), the plain host step loop, the
// batched persistent launch, endpoint de-duplication and the serving loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "homotopy.h"
#include "hp_internal.hpp"
#include "hp_jit.hpp"

using hp::DevSys;
using hp::DevTerm;
using hp::KArgs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(HP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Device allocation owned by the library.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int alloc(size_t b) {
    if (b <= bytes && p) return HP_OK;
    release();
    if (b == 0) return HP_OK;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(e == hipErrorOutOfMemory ? HP_E_OOM : HP_E_DEVICE,
                  std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    bytes = b;
    return HP_OK;
  }
  template <class T>
  T *as() const { return (T *)p; }
};

// ---------------------------------------------------------------------------
// System checks and packing
// ---------------------------------------------------------------------------

struct SysInfo {
  int n = 0;
  int emax = 1;
  int kmax = 0;
  std::vector<int32_t> deg;
  int64_t paths = 0;
};

int check_system(const hp_system *f, SysInfo &info) {
  if (!f) return fail(HP_E_INVALID_ARG, "system is NULL");
  if (f->n < 1 || f->n > HP_MAX_N)
    return fail(HP_E_UNSUPPORTED_N, "n = " + std::to_string(f->n) + " outside 1.." +
                                        std::to_string(HP_MAX_N));
  if (f->n_terms < 1 || !f->eq_ptr || !f->coeff || !f->exps)
    return fail(HP_E_INVALID_ARG, "system has no terms or a NULL array");
  const int n = f->n;
  if (f->eq_ptr[0] != 0 || f->eq_ptr[n] != f->n_terms)
    return fail(HP_E_INVALID_ARG, "eq_ptr must start at 0 and end at n_terms");
  info = SysInfo();
  info.n = n;
  info.deg.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    if (f->eq_ptr[i + 1] < f->eq_ptr[i]) return fail(HP_E_INVALID_ARG, "eq_ptr not monotone");
    for (int t = f->eq_ptr[i]; t < f->eq_ptr[i + 1]; ++t) {
      int d = 0, k = 0;
      for (int j = 0; j < n; ++j) {
        int e = f->exps[(size_t)t * n + j];
        if (e > HP_MAX_EXPONENT)
          return fail(HP_E_INVALID_ARG, "exponent above " + std::to_string(HP_MAX_EXPONENT));
        if (e > 0) {
          ++k;
          info.emax = std::max(info.emax, e);
        }
        d += e;
      }
      const double cr = f->coeff[t].re, ci = f->coeff[t].im;
      if (!std::isfinite(cr) || !std::isfinite(ci))
        return fail(HP_E_INVALID_ARG, "non-finite coefficient");
      info.kmax = std::max(info.kmax, k);
      info.deg[i] = std::max(info.deg[i], d);
    }
    if (info.deg[i] < 1)
      return fail(HP_E_INVALID_ARG, "equation " + std::to_string(i) + " has degree 0");
  }
  int64_t p = 1;
  for (int i = 0; i < n; ++i) {
    if (p > ((int64_t)1 << 62) / info.deg[i]) return fail(HP_E_INVALID_ARG, "too many paths");
    p *= info.deg[i];
  }
  info.paths = p;
  return HP_OK;
}

int check_tol(const hp_tolerances *t) {
  if (!t) return HP_OK;
  auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
  if (!pos(t->h_init) || !pos(t->h_max) || !(t->h_min >= 0.0) || !pos(t->div_radius) ||
      !(t->tol_residual >= 0.0) || !(t->tol_corr >= 0.0) || !(t->tol_final >= 0.0))
    return fail(HP_E_INVALID_ARG, "tolerances must be finite and positive");
  if (t->max_steps < 0 || t->max_steps > 100000000 || t->max_newton < 1 ||
      t->max_newton > 64 || t->max_newton_final < 1 || t->max_newton_final > 64)
    return fail(HP_E_INVALID_ARG, "iteration limits out of range");
  return HP_OK;
}

hp::DevTol dev_tol(const hp_tolerances &t) {
  hp::DevTol d;
  d.tol_residual = t.tol_residual;
  d.tol_corr = t.tol_corr;
  d.tol_final = t.tol_final;
  d.div_radius = t.div_radius;
  d.h_init = t.h_init;
  d.h_min = t.h_min;
  d.h_max = t.h_max;
  d.max_steps = t.max_steps;
  d.max_newton = t.max_newton;
  d.max_newton_final = t.max_newton_final;
  d.pad = 0;
  return d;
}

// Host image of the device system tables of one launch.
struct Packed {
  std::vector<DevTerm> terms;
  std::vector<int32_t> kp;
  std::vector<double2> roots;
  std::vector<DevSys> sys;
  std::vector<double2> dense;  // dense coefficient tables (dense kernel)
  int nl = 1, nmin = HP_MAX_N, emax = 1, kmax = 0;
  bool general = false;  // a general start system or explicit start points
  bool dense_ok = true;  // every system has a dense table
  double dense_fill = 1.0;  // smallest terms / table entries over the systems
  // workgroup LDS bytes of the n_max group variant: largest over the
  // systems, with or without the term tables staged in LDS
  size_t lds(int nmax, bool stage = true) const {
    size_t b = 0;
    for (const DevSys &d : sys)
      b = std::max(b, hp::system_lds_bytes(nmax, d.n, d.emax, d.n_terms, stage));
    return b;
  }
};

// Appends system f (already checked, info from check_system).
// Appends the terms of s (sorted by factor count, equation in byte 15) to
// P.terms and its kKSlots block to P.kp; returns the block's index.
int32_t pack_terms(Packed &P, const hp_system *f, int32_t term_base) {
  const int n = f->n;
  std::vector<std::pair<int, int>> order;  // (k, term)
  std::vector<int> eq_of(f->n_terms);
  for (int i = 0; i < n; ++i)
    for (int t = f->eq_ptr[i]; t < f->eq_ptr[i + 1]; ++t) {
      int k = 0;
      for (int j = 0; j < n; ++j) k += f->exps[(size_t)t * n + j] > 0;
      order.push_back({k, t});
      eq_of[t] = i;
    }
  std::stable_sort(order.begin(), order.end(),
                   [](const std::pair<int, int> &a, const std::pair<int, int> &b) {
                     return a.first < b.first;
                   });
  int32_t kp[hp::kKSlots];
  size_t pos = 0;
  for (int k = 0; k <= HP_MAX_N; ++k) {
    const size_t cls = P.terms.size();
    kp[k] = (int32_t)cls - term_base;
    while (pos < order.size() && order[pos].first == k) {
      const int t = order[pos].second;
      DevTerm T;
      std::memset(&T, 0, sizeof(T));
      T.cre = f->coeff[t].re;
      T.cim = f->coeff[t].im;
      uint8_t bytes[16] = {0};
      bytes[0] = (uint8_t)k;
      int m = 0;
      for (int j = 0; j < n; ++j) {
        const int e = f->exps[(size_t)t * n + j];
        if (e > 0) bytes[1 + m++] = (uint8_t)(j | (e << 4));
      }
      bytes[15] = (uint8_t)eq_of[t];
      std::memcpy(T.w, bytes, 16);
      P.terms.push_back(T);
      ++pos;
    }
    // flag the chunks of this class whose terms all lie in one equation
    for (size_t c0 = cls; c0 < P.terms.size(); c0 += (size_t)n) {
      const size_t c1 = std::min(P.terms.size(), c0 + (size_t)n);
      bool uni = true;
      for (size_t i = c0 + 1; i < c1; ++i) uni = uni && P.terms[i].w[3] >> 24 == P.terms[c0].w[3] >> 24;
      if (uni)
        for (size_t i = c0; i < c1; ++i) P.terms[i].w[0] |= hp::kChunkUniform;
    }
  }
  kp[HP_MAX_N + 1] = (int32_t)P.terms.size() - term_base;
  const int32_t block = (int32_t)P.kp.size();
  P.kp.insert(P.kp.end(), kp, kp + hp::kKSlots);
  return block;
}

// Dense table of f for the dense kernel (n <= kDenseMaxN, every equation of
// total degree <= kDenseMaxDeg), appended to P.dense with its offsets in d;
// false when f does not qualify.  Entry order: the kernel's loops (constant;
// x_a; x_a x_b, a <= b; x_a x_b x_c, a <= b <= c; a outermost).
bool pack_dense(Packed &P, const hp_system *f, const SysInfo &info, DevSys &d) {
  const int n = f->n;
  if (n > hp::kDenseWideMaxN) return false;
  for (int i = 0; i < n; ++i)
    if (info.deg[i] > hp::kDenseMaxDeg) return false;
  const int nq = n * (n + 1) / 2, nc = n * (n + 1) * (n + 2) / 6;
  std::vector<int> qidx((size_t)n * n, -1), cidx((size_t)n * n * n, -1);
  int qi = 1 + n, ci = 1 + n + nq;
  for (int a = 0; a < n; ++a)
    for (int b = a; b < n; ++b) {
      qidx[(size_t)a * n + b] = qi++;
      for (int c = b; c < n; ++c) cidx[((size_t)a * n + b) * n + c] = ci++;
    }
  const size_t base = P.dense.size();
  d.dense_base = (int32_t)base;
  size_t entries = 0;
  for (int i = 0; i < n; ++i) {
    const int di = info.deg[i];
    const size_t size = 1 + n + (di >= 2 ? nq : 0) + (di >= 3 ? nc : 0);
    const size_t eq0 = P.dense.size();
    d.dense_off[i] = (int32_t)(eq0 - base);
    P.dense.resize(eq0 + size, make_double2(0.0, 0.0));
    entries += size;
    for (int t = f->eq_ptr[i]; t < f->eq_ptr[i + 1]; ++t) {
      int v[hp::kDenseMaxDeg], td = 0;  // variables of the monomial, ascending
      for (int j = 0; j < n; ++j)
        for (int e = 0; e < f->exps[(size_t)t * n + j]; ++e) v[td++] = j;
      const int pos = td == 0 ? 0
                    : td == 1 ? 1 + v[0]
                    : td == 2 ? qidx[(size_t)v[0] * n + v[1]]
                              : cidx[((size_t)v[0] * n + v[1]) * n + v[2]];
      P.dense[eq0 + pos].x += f->coeff[t].re;
      P.dense[eq0 + pos].y += f->coeff[t].im;
    }
  }
  P.dense_fill = std::min(P.dense_fill, (double)f->n_terms / (double)entries);
  return true;
}

// f's terms in equation order for the end game (appended to P.terms after
// the tracking kernels' tables; offsets in d.eg_base / d.eg_ptr), each
// term's word holding its dense exponent vector, 4 bits per variable.
void pack_eq_order(Packed &P, const hp_system *f, DevSys &d) {
  const int n = f->n;
  d.eg_base = (int32_t)P.terms.size();
  for (int i = 0; i < n; ++i) {
    d.eg_ptr[i] = (int32_t)P.terms.size() - d.eg_base;
    for (int t = f->eq_ptr[i]; t < f->eq_ptr[i + 1]; ++t) {
      DevTerm T;
      std::memset(&T, 0, sizeof(T));
      T.cre = f->coeff[t].re;
      T.cim = f->coeff[t].im;
      // exponent of variable j in bits 4j .. 4j+3 (exponents are <= 15)
      uint64_t nib = 0;
      for (int j = 0; j < n; ++j) nib |= (uint64_t)f->exps[(size_t)t * n + j] << (4 * j);
      T.w[0] = (uint32_t)nib;
      T.w[1] = (uint32_t)(nib >> 32);
      T.w[3] = (uint32_t)i << 24;
      P.terms.push_back(T);
    }
  }
  d.eg_ptr[n] = (int32_t)P.terms.size() - d.eg_base;
}

void pack_append(Packed &P, const hp_system *f, const SysInfo &info, hp_c64 gamma,
                 int64_t queue_len, int64_t out_path_base, int64_t out_x_base,
                 const int64_t *dev_ids, const hp_system *g = nullptr, int g_emax = 0,
                 const double2 *dev_start = nullptr) {
  const int n = f->n;
  DevSys d;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.emax = info.emax;
  d.eq_base = (int32_t)P.kp.size();
  d.root_base = (int32_t)P.roots.size();
  d.term_base = (int32_t)P.terms.size();
  d.n_terms = f->n_terms;
  int64_t radix = 1;
  int roff = 0;
  for (int i = 0; i < n; ++i) {
    d.deg[i] = info.deg[i];
    d.radix[i] = radix;
    radix *= info.deg[i];
    d.root_off[i] = roff;
    for (int k = 0; k < info.deg[i]; ++k) {
      const double a = 2.0 * M_PI * (double)k / (double)info.deg[i];
      P.roots.push_back(make_double2(std::cos(a), std::sin(a)));
    }
    roff += info.deg[i];
  }
  d.gre = gamma.re;
  d.gim = gamma.im;
  d.n_paths = queue_len;
  d.out_path_base = out_path_base;
  d.out_x_base = out_x_base;
  d.ids = dev_ids;
  // all terms of the system sorted by factor count (stable), equation in byte 15
  const int32_t fblock = pack_terms(P, f, d.term_base);
  (void)fblock;
  if (g) {
    d.g_term_base = (int32_t)P.terms.size();
    d.g_n_terms = g->n_terms;
    d.g_eq_base = pack_terms(P, g, d.g_term_base);
    d.emax = std::max(d.emax, g_emax);
  }
  d.start = dev_start;
  pack_eq_order(P, f, d);
  if (g || dev_start || !pack_dense(P, f, info, d)) P.dense_ok = false;
  P.sys.push_back(d);
  P.nl = std::max(P.nl, n);
  P.nmin = std::min(P.nmin, n);
  P.emax = std::max(P.emax, d.emax);
  P.general = P.general || g || dev_start;
  P.kmax = std::max(P.kmax, info.kmax);
}

// Device copy of a Packed image.
// Pinned host memory (hipHostMalloc), grow-only like DevBuf.
struct HostBuf {
  void *p = nullptr;
  size_t bytes = 0;
  HostBuf() = default;
  HostBuf(const HostBuf &) = delete;
  HostBuf &operator=(const HostBuf &) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  int alloc(size_t b) {
    if (b <= bytes && p) return HP_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, std::max<size_t>(b, 64), hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(HP_E_OOM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    bytes = std::max<size_t>(b, 64);
    return HP_OK;
  }
};

struct DevTables {
  DevBuf tcoef, tmeta, kp, roots, sys, qhead, dcoef, egblk;
  // end-game blocks of a multi-system launch, grouped by n: the blocks of
  // the systems with n unknowns are eg_first[n] .. eg_first[n+1]-1 of egblk
  int eg_first[HP_MAX_N + 2] = {};
  // The system descriptors and the end-game block table (both depend on the
  // queue lengths); synchronous when sync.
  int upload_sys(const Packed &P, hipStream_t s, bool sync) {
    int rc;
    std::vector<int2> blk;
    for (const DevSys &d : P.sys)
      if (d.n_paths > INT32_MAX - hp::kLanes)
        return fail(HP_E_INVALID_ARG, "too many paths for one system of a batch");
    // the end game's list of system k starts where its first block's
    // entries would (one system: at 0)
    std::vector<DevSys> sysv(P.sys);
    for (int n = 1; n <= HP_MAX_N; ++n) {
      eg_first[n] = (int)blk.size();
      for (size_t k = 0; k < P.sys.size(); ++k)
        if (P.sys[k].n == n && P.sys.size() > 1) {
          sysv[k].eg_list_base = (int64_t)blk.size() * hp::kLanes;
          for (int64_t q = 0; q < P.sys[k].n_paths; q += hp::kLanes)
            blk.push_back(make_int2((int)k, (int)q));
        }
    }
    eg_first[HP_MAX_N + 1] = (int)blk.size();
    if ((rc = egblk.alloc(std::max<size_t>(1, blk.size()) * sizeof(int2)))) return rc;
    if (!blk.empty())
      HIP_TRY(hipMemcpyAsync(egblk.p, blk.data(), blk.size() * sizeof(int2),
                             hipMemcpyHostToDevice, s));
    if ((rc = sys.alloc(std::max<size_t>(1, P.sys.size()) * sizeof(DevSys)))) return rc;
    if ((rc = qhead.alloc(std::max<size_t>(1, P.sys.size()) * sizeof(unsigned long long)))) return rc;
    HIP_TRY(hipMemcpyAsync(sys.p, sysv.data(), sysv.size() * sizeof(DevSys),
                           hipMemcpyHostToDevice, s));
    if (sync) HIP_TRY(hipStreamSynchronize(s));
    return HP_OK;
  }
  int upload(const Packed &P, hipStream_t s) {
    int rc;
    if ((rc = upload_sys(P, s, false))) return rc;
    const size_t nt = std::max<size_t>(1, P.terms.size());
    if ((rc = dcoef.alloc(std::max<size_t>(1, P.dense.size()) * sizeof(double2)))) return rc;
    if (!P.dense.empty())
      HIP_TRY(hipMemcpyAsync(dcoef.p, P.dense.data(), P.dense.size() * sizeof(double2),
                             hipMemcpyHostToDevice, s));
    if ((rc = tcoef.alloc(nt * sizeof(double2)))) return rc;
    if ((rc = tmeta.alloc(nt * sizeof(uint4)))) return rc;
    if ((rc = kp.alloc(std::max<size_t>(1, P.kp.size()) * sizeof(int32_t)))) return rc;
    if ((rc = roots.alloc(std::max<size_t>(1, P.roots.size()) * sizeof(double2)))) return rc;
    std::vector<double2> coef(P.terms.size());
    std::vector<uint4> meta(P.terms.size());
    for (size_t i = 0; i < P.terms.size(); ++i) {
      coef[i] = make_double2(P.terms[i].cre, P.terms[i].cim);
      std::memcpy(&meta[i], P.terms[i].w, sizeof(uint4));
    }
    HIP_TRY(hipMemcpyAsync(tcoef.p, coef.data(), coef.size() * sizeof(double2),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(tmeta.p, meta.data(), meta.size() * sizeof(uint4),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(kp.p, P.kp.data(), P.kp.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(roots.p, P.roots.data(), P.roots.size() * sizeof(double2),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HP_OK;
  }
};

// ---------------------------------------------------------------------------
// Kernel variant choice and autotune cache
// ---------------------------------------------------------------------------

int nmax_for(int n) {
  for (int v : hp::kNmaxVariants)
    if (v >= n) return v;
  return -1;
}

// Kernel variant codes: n_max (4, 8, 10, 12) for the group kernels (n lanes
// per path), 100 + n_max for the lane kernels with 64 paths per wavefront,
// 200 + n_max for those with 32, 300 + n for the kernel specialised to
// the plan's system (one path per lane, compiled at run time), and 400 for
// the dense kernel (one path per lane, systems of total degree <= 3).
struct Kv {
  int code = 0;
  bool lanes = false;
  bool spec = false;  // specialised to the plan's system (compiled at run time)
  bool dense = false;  // the dense kernel (any n <= kDenseMaxN, degree <= 3)
  int nmax = 0;
  int pw = 0;  // lane kernels: paths per wavefront
  const hp::SpecModule *sm = nullptr;  // spec: the loaded module
  // launch shape (tuning choices): paths per wavefront of a specialised or
  // dense kernel (0: 64), resident wavefronts per SIMD the launch is capped
  // at (0: as many as fit)
  int lp = 0, wps = 0;
  // spec in the coefficient-parameter form: its (cf, cg, gamma cg - cf) table
  const double2 *pcoef = nullptr;
};

constexpr int kDenseCode = 400;

bool kv_decode(int code, Kv &k) {
  k = Kv{};
  k.code = code;
  for (int v : hp::kNmaxVariants)
    if (code == v) {
      k.nmax = v;
      return true;
    }
  for (const hp::LaneVariant &v : hp::kLaneVariants)
    if (code == (v.pw == 64 ? 100 : 200) + v.n) {
      k.lanes = true;
      k.nmax = v.n;  // lane kernels are compiled for one exact n
      k.pw = v.pw;
      return true;
    }
  if (code > 300 && code <= 300 + hp::kSpecMaxN) {
    k.spec = true;
    k.nmax = code - 300;  // one path per lane, one exact system
    k.pw = hp::kLanes;
    return true;
  }
  if (code == kDenseCode || (code > kDenseCode + hp::kDenseMaxN &&
                             code <= kDenseCode + hp::kDenseWideMaxN)) {
    k.dense = true;
    k.nmax = code == kDenseCode ? hp::kDenseMaxN : code - kDenseCode;
    k.pw = hp::kLanes;
    return true;
  }
  return false;
}

// Dense kernel for the systems of P: 400 (k_dense) when every n <= kDenseMaxN,
// 400 + n (k_dense_n<11>, k_dense_n<12>) when they all have that one larger n,
// else 0.
int dense_code_for(const Packed &P) {
  if (!P.dense_ok) return 0;
  if (P.nl <= hp::kDenseMaxN) return kDenseCode;
  if (P.nmin == P.nl && P.nl <= hp::kDenseWideMaxN) return kDenseCode + P.nl;
  return 0;
}

// True when kernel k runs the systems of P.
bool dense_fits(const Kv &k, const Packed &P) {
  return k.dense && P.dense_ok &&
         (k.code == kDenseCode ? P.nl <= hp::kDenseMaxN : (P.nmin == k.nmax && P.nl == k.nmax));
}

// The dense kernel is the default for launches whose systems all have dense
// tables filled to at least a quarter (sparser systems evaluate faster term
// by term).
int dense_preferred(const Packed &P) { return P.dense_fill >= 0.25 ? dense_code_for(P) : 0; }

// Variants that can run systems of up to n unknowns and exponents up to
// emax within max_lds bytes of LDS (group kernels: checked per system).
std::vector<int> kv_candidates(int n, int emax, size_t max_lds) {
  std::vector<int> out;
  for (const hp::LaneVariant &v : hp::kLaneVariants)
    if (v.n == n && hp::lanes_lds_bytes(v.n, v.pw, emax) <= max_lds)
      out.push_back((v.pw == 64 ? 100 : 200) + v.n);
  for (int v : hp::kNmaxVariants)
    if (v >= n) out.push_back(v);
  return out;
}

// Default among the compiled-ahead kernels for sparse systems: the group
// kernel of the smallest n_max >= n (faster than the lane kernels on the
// measured workloads, which stay autotuner candidates).
int kv_default(int n) { return nmax_for(n); }

// A tuned launch: kernel variant code, paths per wavefront (lp) and
// wavefronts per SIMD (wps) as in Kv.
struct TuneVal {
  int code = 0, lp = 0, wps = 0;
};

std::mutex g_tune_mu;
std::map<std::string, TuneVal> g_tune_mem;

std::string tune_path() {
  const char *p = std::getenv("HP_TUNE_CACHE");
  return p ? std::string(p) : std::string();
}

// Cache key of one system's shape: device (gfx950 and its compute units), n,
// terms, largest exponent and largest factor count of a term.
std::string tune_key(int cus, const SysInfo &info, int n_terms) {
  std::ostringstream o;
  o << "gfx950:cu" << cus << ":n" << info.n << ":t" << n_terms << ":e" << info.emax << ":k"
    << info.kmax;
  return o.str();
}

// Cache key of a batch: the number of systems, their range of n, all their
// terms, the largest exponent and factor count, and whether every system
// has a dense table.
std::string tune_key_batch(int cus, const Packed &P, int64_t total_terms) {
  std::ostringstream o;
  o << "gfx950:cu" << cus << ":batch:s" << P.sys.size() << ":n" << P.nmin << "-" << P.nl << ":t"
    << total_terms << ":e" << P.emax << ":k" << P.kmax << ":d" << (P.dense_ok ? 1 : 0);
  return o.str();
}

// Lines "key code [lp wps]" of the cache file; later lines win.
bool tune_lookup(const std::string &key, TuneVal &out) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune_mem.find(key);
  if (it == g_tune_mem.end()) {
    std::string path = tune_path();
    if (path.empty()) return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      TuneVal v;
      if (!(ls >> k >> v.code)) continue;
      if (!(ls >> v.lp >> v.wps)) v.lp = v.wps = 0;
      g_tune_mem[k] = v;
    }
    it = g_tune_mem.find(key);
    if (it == g_tune_mem.end()) return false;
  }
  out = it->second;
  return true;
}

void tune_store(const std::string &key, const TuneVal &v) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune_mem[key] = v;
  std::string path = tune_path();
  if (path.empty()) return;
  std::ofstream out(path, std::ios::app);
  out << key << " " << v.code << " " << v.lp << " " << v.wps << "\n";
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

// Workspace of the device duplicate scan (grown on demand).
struct DupWork {
  DevBuf keys, ids, keys_sorted, ids_sorted, temp, counts, pairs;
  long long cap = 0, max_pairs = 0;
  size_t temp_bytes = 0;
  int reserve(long long want_cap, long long want_pairs) {
    int rc;
    if (want_cap > cap) {
      cap = std::max<long long>(want_cap, 1 << 12);
      temp_bytes = hp_dup_sort_temp_bytes(cap);
      if ((rc = keys.alloc(cap * sizeof(double))) || (rc = ids.alloc(cap * sizeof(long long))) ||
          (rc = keys_sorted.alloc(cap * sizeof(double))) ||
          (rc = ids_sorted.alloc(cap * sizeof(long long))) || (rc = temp.alloc(temp_bytes)))
        return rc;
    }
    if (want_pairs > max_pairs) {
      max_pairs = std::max<long long>(want_pairs, 1 << 12);
      if ((rc = pairs.alloc(2 * max_pairs * sizeof(long long)))) return rc;
    }
    return counts.alloc(2 * sizeof(unsigned long long));
  }
};

struct hp_context {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evm = nullptr;  // evm: tracking kernel done
  DupWork dup;
  hp_timing last{};
  int cus = 0;
  size_t max_lds = 0;
  // plans and servers made from this context, and whether the caller has
  // destroyed it: the context is released when both no child is left and
  // the caller has destroyed it, so the order of destruction is free
  int children = 0;
  bool closed = false;
};

namespace {

std::mutex g_ctx_mu;

void context_release(hp_context *ctx) {
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->evm) (void)hipEventDestroy(ctx->evm);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

void context_adopt(hp_context *ctx) {
  std::lock_guard<std::mutex> g(g_ctx_mu);
  ++ctx->children;
}

// A child of ctx is gone; releases ctx if it was the last one and the
// caller has destroyed ctx already.
void context_orphan(hp_context *ctx) {
  bool last;
  {
    std::lock_guard<std::mutex> g(g_ctx_mu);
    last = --ctx->children == 0 && ctx->closed;
  }
  if (last) context_release(ctx);
}

}  // namespace

// Device list of the paths a single-system end game refines (a plan's).
struct EgList {
  DevBuf list, count;
  bool ready = false;  // sized and zeroed for the next end game (eg_prepare)
};

struct hp_plan {
  hp_context *ctx = nullptr;
  SysInfo info;
  int n_terms = 0;
  Packed P;
  DevTables dev;
  hp_tolerances tol{};
  hp_c64 gamma{};
  Kv kv;  // kernel variant and launch shape
  hp_tune_choice tune{};  // the autotuner's record (zero: not tuned)
  bool spec_default = false;  // default variant: the specialised kernel where it applies
  DevBuf start_dev;  // explicit start points [n_start][n] (general plans)
  DevBuf pcoef;      // (cf, cg, gamma cg - cf) per term: coefficient-parameter plans
  EgList eg;         // the end game's list of paths to refine
  // plain-mode state
  DevBuf px0, pt, ph, piv, pactive;
  DevBuf ids_scratch;
};

extern "C" {

const char *hp_last_error(void) { return g_err.c_str(); }

void hp_default_tolerances(hp_tolerances *t) {
  if (!t) return;
  t->tol_residual = 1e-10;
  t->tol_corr = 1e-8;
  t->tol_final = 1e-13;
  t->div_radius = 1e8;
  t->h_init = 0.01;
  t->h_min = 1e-13;
  t->h_max = 0.1;
  t->max_steps = 10000;
  t->max_newton = 3;
  t->max_newton_final = 6;
}

int hp_context_create(int device, hp_context **out) {
  if (!out) return fail(HP_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return fail(HP_E_INVALID_ARG, "no HIP device " + std::to_string(device));
  HIP_TRY(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(HP_E_DEVICE, std::string("libhomotopy is built for gfx950, device is ") +
                                 prop.gcnArchName);
  std::unique_ptr<hp_context> c(new hp_context());
  c->device = device;
  c->cus = prop.multiProcessorCount;
  c->max_lds = prop.sharedMemPerBlock;
  HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  HIP_TRY(hipEventCreate(&c->evm));
  *out = c.release();
  return HP_OK;
}

void hp_context_destroy(hp_context *ctx) {
  if (!ctx) return;
  bool now;
  {
    std::lock_guard<std::mutex> g(g_ctx_mu);
    ctx->closed = true;
    now = ctx->children == 0;
  }
  if (now) context_release(ctx);
}

int hp_last_timing(const hp_context *ctx, hp_timing *out) {
  if (!ctx || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  *out = ctx->last;
  return HP_OK;
}

int64_t hp_path_count(const hp_system *f) {
  SysInfo info;
  if (check_system(f, info) != HP_OK) return -1;
  return info.paths;
}

}  // extern "C"

namespace {

int check_lds(hp_context *ctx, size_t lds) {
  if (lds > ctx->max_lds)
    return fail(HP_E_UNSUPPORTED_N, "workgroup LDS " + std::to_string(lds) +
                                        " B exceeds the device limit");
  return HP_OK;
}

// LDS bytes per workgroup of variant k for the systems of P.
size_t kv_lds(const Kv &k, const Packed &P) {
  if (k.spec || k.dense) return 0;
  return k.lanes ? hp::lanes_lds_bytes(k.nmax, k.pw, P.emax) : P.lds(k.nmax, false);
}

// LDS bytes, resident workgroups per CU and term staging of variant k for
// the systems of P.  Group kernels stage small term tables in LDS unless
// that lowers the number of resident workgroups.
// Paths a wavefront of variant k holds (systems of up to nl unknowns).
int kv_paths_per_wave(const Kv &k, int nl) {
  if ((k.spec || k.dense) && k.lp > 0) return k.lp;
  return (k.lanes || k.spec || k.dense) ? k.pw : hp::kLanes / std::max(1, nl);
}

// The launch shape of variant k in the timing record.
void timing_shape(hp_timing &t, const Kv &k, int nl) {
  t.paths_per_wave = kv_paths_per_wave(k, nl);
  t.lanes_per_path = (k.lanes || k.spec || k.dense) ? 1 : nl;
  t.waves_per_simd = k.wps;
  t.max_n = k.nmax;
  t.variant = k.code;
}

int kv_occupancy(hp_context *ctx, const Kv &k, const Packed &P, size_t *lds, int *per_cu,
                 int *stage, bool sliced = false) {
  *stage = 0;
  if (k.spec) {
    *lds = 0;
    HIP_TRY(hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k.sm->persistent, hp::kLanes, 0));
  } else if (k.dense) {
    *lds = 0;
    if (sliced) {
      if (k.code == kDenseCode) HIP_TRY((hipError_t)hp_dense_sliced_per_cu(per_cu));
      else HIP_TRY((hipError_t)hp_dense_wide_sliced_per_cu(k.nmax, per_cu));
    } else if (k.code == kDenseCode) {
      HIP_TRY((hipError_t)hp_dense_per_cu(per_cu));
    } else if (k.nmax == 11) {
      HIP_TRY((hipError_t)hp_dense11_per_cu(per_cu));
    } else {
      HIP_TRY((hipError_t)hp_dense12_per_cu(per_cu));
    }
  } else if (k.lanes) {
    *lds = kv_lds(k, P);
    int rc = check_lds(ctx, *lds);
    if (rc) return rc;
    HIP_TRY((hipError_t)hp_lanes_per_cu(k.nmax, k.pw, *lds, per_cu));
  } else {
    const size_t ln = P.lds(k.nmax, false), ls = P.lds(k.nmax, true);
    int rc = check_lds(ctx, ln);
    if (rc) return rc;
    int on = 0, os = 0;
    HIP_TRY((hipError_t)hp_max_groups_per_cu(k.nmax, P.general, ln, &on));
    if (ls <= ctx->max_lds) HIP_TRY((hipError_t)hp_max_groups_per_cu(k.nmax, P.general, ls, &os));
    *stage = (ls <= ctx->max_lds && os >= on) ? 1 : 0;
    *lds = *stage ? ls : ln;
    *per_cu = *stage ? os : on;
  }
  if (*per_cu < 1) return fail(HP_E_DEVICE, "kernel variant does not fit on a compute unit");
  return HP_OK;
}

// Default variant of a launch over packed systems (one-shot calls, batches,
// serving requests): the dense kernel when the systems suit it, else the
// group kernel for their widest n.
Kv kv_pick(const Packed &P) {
  Kv k;
  if (const int dc = dense_preferred(P)) kv_decode(dc, k);
  else kv_decode(kv_default(P.nl), k);
  return k;
}

// End game at t = 1 (double-double refinement and residual test) of the
// paths a tracking launch over the systems in `dev` has just ended, on the
// same stream.  total_paths: the queue length of a single-system launch.
// With eg given, the paths to refine are first compacted into its list (per
// n for a multi-system launch), so that the end game's wavefronts are full.
// dense: the launch ran a dense kernel, whose coefficient tables then serve
// the end game too.
// Entries of the end game's lists for a launch over the systems in `dev`:
// per system a list region from its eg_list_base (64 entries per block of
// its queue).
int64_t eg_entries(const DevTables &dev, const Packed &P, int64_t total_paths) {
  if (P.sys.size() == 1) return (total_paths + hp::kLanes - 1) / hp::kLanes * hp::kLanes;
  return (int64_t)dev.eg_first[HP_MAX_N + 1] * hp::kLanes;
}

// Sizes eg's list and zeroes its per-system counters on stream s, ahead of
// the end game of a launch over the systems in `dev`.  launch_endgame does
// this itself unless it has been done; the server does it for all its
// families before any of their kernels runs, since a fill or an allocation
// issued while another stream's persistent kernel holds every compute unit
// waits for that kernel to end.
int eg_prepare(EgList &eg, const DevTables &dev, const Packed &P, int64_t total_paths,
               hipStream_t s) {
  const int64_t entries = eg_entries(dev, P, total_paths);
  eg.ready = false;
  if (entries > 0) {
    int rc;
    if ((rc = eg.list.alloc((size_t)entries * sizeof(long long)))) return rc;
    if ((rc = eg.count.alloc(P.sys.size() * sizeof(unsigned)))) return rc;
    HIP_TRY(hipMemsetAsync(eg.count.p, 0, P.sys.size() * sizeof(unsigned), s));
  }
  eg.ready = true;
  return HP_OK;
}

int launch_endgame(const DevTables &dev, const Packed &P, const KArgs &a, int64_t total_paths,
                   hipStream_t s, EgList *eg = nullptr, bool dense = false) {
  const bool one = P.sys.size() == 1;
  const int64_t single_blocks = (total_paths + hp::kLanes - 1) / hp::kLanes;
  if (one && single_blocks > INT32_MAX) return fail(HP_E_INVALID_ARG, "too many paths for one launch");
  if (eg) {
    if (eg_entries(dev, P, total_paths) == 0) return HP_OK;
    int rc;
    if (!eg->ready && (rc = eg_prepare(*eg, dev, P, total_paths, s))) return rc;
    eg->ready = false;  // the next end game zeroes the counters again
    KArgs b = a;
    b.eg_list = eg->list.as<long long>();
    b.eg_count = eg->count.as<unsigned>();
    if (one) {
      HIP_TRY((hipError_t)hp_launch_eg_select(a, nullptr, (int)single_blocks, eg->list.as<long long>(),
                                              eg->count.as<unsigned>(), s));
      HIP_TRY((hipError_t)hp_launch_endgame(P.sys[0].n, b, nullptr, (int)single_blocks, dense, s));
      return HP_OK;
    }
    HIP_TRY((hipError_t)hp_launch_eg_select(a, dev.egblk.as<int2>(), dev.eg_first[HP_MAX_N + 1],
                                            eg->list.as<long long>(), eg->count.as<unsigned>(), s));
    for (int n = 1; n <= HP_MAX_N; ++n) {
      const int b0 = dev.eg_first[n], b1 = dev.eg_first[n + 1];
      if (b1 > b0)
        HIP_TRY((hipError_t)hp_launch_endgame(n, b, dev.egblk.as<int2>() + b0, b1 - b0, dense, s));
    }
    return HP_OK;
  }
  if (one) {
    HIP_TRY((hipError_t)hp_launch_endgame(P.sys[0].n, a, nullptr, (int)single_blocks, dense, s));
    return HP_OK;
  }
  for (int n = 1; n <= HP_MAX_N; ++n) {
    const int b0 = dev.eg_first[n], b1 = dev.eg_first[n + 1];
    if (b1 > b0)
      HIP_TRY((hipError_t)hp_launch_endgame(n, a, dev.egblk.as<int2>() + b0, b1 - b0, dense, s));
  }
  return HP_OK;
}

// Persistent launch over the systems in `dev` (already uploaded), followed
// by the end game of its paths.  step_budget >= 0 selects the serving form
// of the specialised (the module must be one) and dense kernels, with that
// many steps per wavefront (0: no limit); -1 the plain form.
int launch_persistent(hp_context *ctx, DevTables &dev, const Packed &P, const Kv &k,
                      const hp_tolerances &tol, int64_t total_paths, hp_c64 *endpoints,
                      int32_t *status, hp_path_stats *stats, hipStream_t s, int *groups_out,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, hipEvent_t em = nullptr,
                      int32_t step_budget = -1, EgList *eg = nullptr, bool qhead_zeroed = false) {
  const bool sliced = step_budget >= 0;
  if (sliced && !k.spec && !k.dense) return fail(HP_E_INVALID_ARG, "no serving form of this kernel");
  if (!e0) {  // the context's events: e0 .. em the tracking kernel, em .. e1 the end game
    e0 = ctx->ev0;
    e1 = ctx->ev1;
    em = ctx->evm;
  }
  if (P.nl > k.nmax || (k.lanes && P.nmin != k.nmax) ||
      (k.spec && (P.nl != k.nmax || P.nmin != k.nmax || !k.sm)) || (k.dense && !dense_fits(k, P)))
    return fail(HP_E_INVALID_ARG, "kernel variant does not match the systems' n");
  size_t lds = 0;
  int per_cu = 0, stage = 0;
  int rc = kv_occupancy(ctx, k, P, &lds, &per_cu, &stage, sliced);
  if (rc) return rc;
  // enough wavefronts to hold every path once, at most a full device (or
  // the tuned number of wavefronts per SIMD: 4 SIMDs per CU)
  const int lp = (k.spec || k.dense) ? k.lp : 0;
  const int64_t per_wave = lp ? lp : kv_paths_per_wave(k, P.nl);
  const int64_t want = (total_paths + per_wave - 1) / per_wave;
  const int cap = k.wps > 0 ? std::min(per_cu, 4 * k.wps) : per_cu;
  const int64_t groups = std::min<int64_t>((int64_t)ctx->cus * cap, std::max<int64_t>(1, want));
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sys = dev.sys.as<DevSys>();
  a.n_systems = (int32_t)P.sys.size();
  a.tcoef = dev.tcoef.as<double2>();
  a.tmeta = dev.tmeta.as<uint4>();
  a.eqp = dev.kp.as<int32_t>();
  a.roots = dev.roots.as<double2>();
  a.qhead = dev.qhead.as<unsigned long long>();
  a.endpoints = (double2 *)endpoints;
  a.status = status;
  a.stats = stats;
  a.tol = dev_tol(tol);
  a.stage = stage;
  a.dcoef = dev.dcoef.as<double2>();
  a.step_budget = sliced ? step_budget : 0;
  a.lane_paths = lp;
  a.pcoef = k.pcoef;
  if (!qhead_zeroed)
    HIP_TRY(hipMemsetAsync(dev.qhead.p, 0, P.sys.size() * sizeof(unsigned long long), s));
  HIP_TRY(hipEventRecord(e0, s));
  if (k.spec) {
    void *params[] = {&a};
    HIP_TRY(hipModuleLaunchKernel(k.sm->persistent, (unsigned)groups, 1, 1, hp::kLanes, 1, 1, 0, s,
                                  params, nullptr));
  } else if (k.dense && sliced) {
    if (k.code == kDenseCode) HIP_TRY((hipError_t)hp_launch_dense_sliced(a, (int)groups, s));
    else HIP_TRY((hipError_t)hp_launch_dense_wide_sliced(k.nmax, a, (int)groups, s));
  } else if (k.dense) {
    if (k.code == kDenseCode) HIP_TRY((hipError_t)hp_launch_dense(a, (int)groups, s));
    else if (k.nmax == 11) HIP_TRY((hipError_t)hp_launch_dense11(a, (int)groups, s));
    else HIP_TRY((hipError_t)hp_launch_dense12(a, (int)groups, s));
  } else if (k.lanes) {
    HIP_TRY((hipError_t)hp_launch_lanes(k.nmax, k.pw, a, (int)groups, lds, s));
  } else {
    HIP_TRY((hipError_t)hp_launch_persistent(k.nmax, P.general, a, (int)groups, lds, s));
  }
  if (em) HIP_TRY(hipEventRecord(em, s));
  if ((rc = launch_endgame(dev, P, a, total_paths, s, eg, k.dense))) return rc;
  HIP_TRY(hipEventRecord(e1, s));
  if (groups_out) *groups_out = (int)groups;
  return HP_OK;
}

// A general plan whose start system g has f's support term by term (same
// equations, same monomials in the same order) and explicit start points:
// a coefficient-parameter continuation, which the specialised kernel's
// coefficient-parameter form runs.
bool plan_param(const hp_plan *plan) {
  const Packed &P = plan->P;
  if (!P.general || P.sys.size() != 1) return false;
  const DevSys &d = P.sys[0];
  if (!d.start || d.g_n_terms != d.n_terms || d.n_terms == 0) return false;
  for (int t = 0; t < d.n_terms; ++t)
    if (std::memcmp(P.terms[d.term_base + t].w, P.terms[d.g_term_base + t].w,
                    sizeof(P.terms[0].w)) != 0)
      return false;
  return true;
}

// The plan's system can have a kernel specialised to it.
bool plan_spec_eligible(const hp_plan *plan) {
  const Packed &P = plan->P;
  return (!P.general || plan_param(plan)) && P.sys.size() == 1 &&
         hp::spec_eligible(plan->info.n, P.terms.data() + P.sys[0].term_base, P.sys[0].n_terms);
}

// Generates, compiles (hiprtc; cached per process) and loads the kernel
// specialised to the plan's system; for a coefficient-parameter plan the
// coefficient-parameter form, with its coefficient table uploaded.
int spec_prepare(hp_plan *plan, Kv &k) {
  const Packed &P = plan->P;
  const DevSys &d = P.sys[0];
  const bool param = plan_param(plan);
  const std::string src =
      hp::spec_source(plan->info.n, d.deg, P.terms.data() + d.term_base, d.n_terms, false, param);
  std::string log;
  const int rc = hp::spec_get(plan->ctx->device, src, &k.sm, log);
  if (rc) return fail(HP_E_DEVICE, "specialised kernel: " + std::string(hipGetErrorString((hipError_t)rc)) +
                                       (log.empty() ? "" : "\n" + log));
  if (param) {
    // per term in packed order: f's coefficient, g's, and gamma g - f (the
    // coefficient of -H_t)
    std::vector<double2> tab((size_t)3 * d.n_terms);
    for (int t = 0; t < d.n_terms; ++t) {
      const DevTerm &F = P.terms[d.term_base + t], &G = P.terms[d.g_term_base + t];
      tab[3 * t] = make_double2(F.cre, F.cim);
      tab[3 * t + 1] = make_double2(G.cre, G.cim);
      tab[3 * t + 2] = make_double2(d.gre * G.cre - d.gim * G.cim - F.cre,
                                    d.gre * G.cim + d.gim * G.cre - F.cim);
    }
    int r = plan->pcoef.alloc(tab.size() * sizeof(double2));
    if (r) return r;
    HIP_TRY(hipMemcpy(plan->pcoef.p, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice));
    k.pcoef = plan->pcoef.as<double2>();
  }
  return HP_OK;
}

int plan_variant(hp_plan *plan, int code) {
  if (code == 0) {
    const int dc = dense_preferred(plan->P);
    code = (plan->spec_default && plan_spec_eligible(plan)) ? 300 + plan->info.n
           : dc ? dc
                : kv_default(plan->info.n);
  }
  Kv k;
  if (!kv_decode(code, k) || k.nmax < plan->info.n ||
      ((k.lanes || k.spec || (k.dense && k.code != kDenseCode)) && k.nmax != plan->info.n))
    return fail(HP_E_INVALID_ARG, "no compiled kernel variant " + std::to_string(code) +
                                      " for n = " + std::to_string(plan->info.n));
  if ((k.lanes || k.dense || (k.spec && !plan_param(plan))) && plan->P.general)
    return fail(HP_E_INVALID_ARG, "lane kernels track the total-degree start system only "
                                  "(the specialised kernel also a start system on f's support)");
  if (k.dense && !dense_fits(k, plan->P))
    return fail(HP_E_INVALID_ARG, "the dense kernels take n <= " +
                                      std::to_string(hp::kDenseWideMaxN) +
                                      " and equations of total degree <= " +
                                      std::to_string(hp::kDenseMaxDeg));
  if (k.spec) {
    if (!plan_spec_eligible(plan))
      return fail(HP_E_INVALID_ARG, "system too large for a specialised kernel");
    int rc = spec_prepare(plan, k);
    if (rc) return rc;
  }
  int rc = check_lds(plan->ctx, kv_lds(k, plan->P));
  if (rc) return rc;
  plan->kv = k;
  return HP_OK;
}

int track_plain(hp_plan *plan, const int64_t *ids, int64_t n_paths, hp_c64 *endpoints,
                int32_t *status, hp_path_stats *stats, hipStream_t s) {
  hp_context *ctx = plan->ctx;
  const int n = plan->info.n;
  int rc;
  if ((rc = plan->px0.alloc((size_t)n * n_paths * sizeof(double2)))) return rc;
  if ((rc = plan->pt.alloc((size_t)n_paths * sizeof(double)))) return rc;
  if ((rc = plan->ph.alloc((size_t)n_paths * sizeof(double)))) return rc;
  if ((rc = plan->piv.alloc((size_t)8 * n_paths * sizeof(int32_t)))) return rc;
  if ((rc = plan->pactive.alloc(sizeof(unsigned int)))) return rc;
  // the dense kernel has no plain form: plain calls of a dense plan run the
  // group kernel
  Kv k = plan->kv;
  if (k.dense) kv_decode(nmax_for(n), k);
  size_t lds = 0;
  int per_cu = 0, stage = 0;
  if ((rc = kv_occupancy(ctx, k, plan->P, &lds, &per_cu, &stage))) return rc;
  // system descriptor with this call's queue and ids
  DevSys d = plan->P.sys[0];
  d.n_paths = n_paths;
  d.ids = ids;
  HIP_TRY(hipMemcpyAsync(plan->dev.sys.p, &d, sizeof(d), hipMemcpyHostToDevice, s));
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sys = plan->dev.sys.as<DevSys>();
  a.n_systems = 1;
  a.tcoef = plan->dev.tcoef.as<double2>();
  a.tmeta = plan->dev.tmeta.as<uint4>();
  a.eqp = plan->dev.kp.as<int32_t>();
  a.roots = plan->dev.roots.as<double2>();
  a.endpoints = (double2 *)endpoints;
  a.status = status;
  a.stats = stats;
  a.tol = dev_tol(plan->tol);
  a.ps.x0 = plan->px0.as<double2>();
  a.ps.t = plan->pt.as<double>();
  a.ps.h = plan->ph.as<double>();
  a.ps.iv = plan->piv.as<int32_t>();
  a.ps.P = n_paths;
  a.ps.active = plan->pactive.as<unsigned int>();
  a.stage = stage;
  a.pcoef = k.pcoef;
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  HIP_TRY((hipError_t)hp_launch_plain_init(a, s));
  const int64_t per_wave = (k.lanes || k.spec) ? k.pw : hp::kLanes / n;
  const int wgs = (int)((n_paths + per_wave - 1) / per_wave);
  // every path ends within max_steps + 1 attempts plus the final Newton
  const int64_t max_launches = (int64_t)plan->tol.max_steps + 4;
  int64_t launches = 0;
  unsigned int active = 1;
  while (active > 0 && launches < max_launches) {
    HIP_TRY(hipMemsetAsync(plan->pactive.p, 0, sizeof(unsigned int), s));
    if (k.spec) {
      void *params[] = {&a};
      HIP_TRY(hipModuleLaunchKernel(k.sm->plain, (unsigned)wgs, 1, 1, hp::kLanes, 1, 1, 0, s,
                                    params, nullptr));
    } else if (k.lanes) {
      HIP_TRY((hipError_t)hp_launch_lanes_plain(k.nmax, k.pw, a, wgs, lds, s));
    } else {
      HIP_TRY((hipError_t)hp_launch_plain_step(k.nmax, plan->P.general, a, wgs, lds, s));
    }
    HIP_TRY(hipMemcpyAsync(&active, plan->pactive.p, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    ++launches;
  }
  HIP_TRY(hipEventRecord(ctx->evm, s));
  if (active == 0 && (rc = launch_endgame(plan->dev, plan->P, a, n_paths, s, &plan->eg))) return rc;
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  ctx->last.launches = launches;
  ctx->last.groups = wgs;
  if (active > 0) return fail(HP_E_DEVICE, "plain tracker did not finish");
  return HP_OK;
}

// Launch shapes of variant k to time: paths per wavefront 64 or 32 for the
// specialised and dense kernels, and every cap on the wavefronts per SIMD
// that binds (below the occupancy of the variant).
std::vector<Kv> tune_shapes(hp_context *ctx, const Kv &k, const Packed &P) {
  std::vector<Kv> out;
  size_t lds = 0;
  int per_cu = 0, stage = 0;
  if (kv_occupancy(ctx, k, P, &lds, &per_cu, &stage) != HP_OK) return out;
  const int max_wps = (per_cu + 3) / 4;
  for (int lp : (k.spec || k.dense) ? std::vector<int>{0, 32} : std::vector<int>{0})
    for (int wps = 0; wps < max_wps; ++wps) {
      Kv v = k;
      v.lp = lp;
      v.wps = wps;
      out.push_back(v);
    }
  return out;
}

// Times candidate launch shapes with run(k) (the kernel milliseconds of one
// launch over the sample the caller set up; the second of two runs counts)
// and returns the fastest; default_ms: the time of `def`'s shape.
template <class Run>
int tune_pick(const std::vector<Kv> &cands, const Kv &def, Run run, Kv &best_k, hp_tune_choice &c) {
  double best = 1e300;
  c.ms_default = -1.0;
  c.candidates = 0;
  for (const Kv &k : cands) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      const int rc = run(k, ms);
      if (rc) return rc;
    }
    ++c.candidates;
    if (k.code == def.code && k.lp == def.lp && k.wps == def.wps) c.ms_default = ms;
    if (ms < best) {
      best = ms;
      best_k = k;
    }
  }
  c.ms = best;
  return HP_OK;
}

// Packs a batch (offsets from hp_batch_layout); total_terms: all terms.
int pack_batch(const hp_system *fs, int32_t n_systems, const hp_c64 *gammas,
               std::vector<int64_t> &po, std::vector<int64_t> &xo, Packed &P, int64_t &total_terms) {
  int rc = hp_batch_layout(fs, n_systems, po.data(), xo.data());
  if (rc) return rc;
  total_terms = 0;
  for (int s = 0; s < n_systems; ++s) {
    SysInfo info;
    check_system(&fs[s], info);
    pack_append(P, &fs[s], info, gammas[s], info.paths, po[s], xo[s], nullptr);
    total_terms += fs[s].n_terms;
  }
  return HP_OK;
}

// Variant `code` runs every system of the batch P (dense or group kernels).
bool batch_variant_ok(hp_context *ctx, const Packed &P, int code, Kv &k) {
  if (!kv_decode(code, k) || k.lanes || k.spec) return false;
  if (k.dense) return dense_fits(k, P);
  return k.nmax >= P.nl && check_lds(ctx, P.lds(k.nmax, false)) == HP_OK;
}

void choice_from_kv(hp_tune_choice &c, const Kv &k, int nl) {
  hp_timing t{};
  timing_shape(t, k, nl);
  c.variant = k.code;
  c.paths_per_wave = t.paths_per_wave;
  c.lanes_per_path = t.lanes_per_path;
  c.waves_per_simd = k.wps;
}

// Checks a cached or forced launch shape against variant k.
bool shape_ok(const Kv &k, int lp, int wps) {
  return wps >= 0 && wps <= 64 && (lp == 0 || ((k.spec || k.dense) && lp >= 1 && lp <= hp::kLanes));
}

int autotune(hp_plan *plan) {
  hp_context *ctx = plan->ctx;
  const std::string key = tune_key(ctx->cus, plan->info, plan->n_terms);
  plan->tune = hp_tune_choice{};
  TuneVal cv;
  if (tune_lookup(key, cv) && plan_variant(plan, cv.code) == HP_OK && shape_ok(plan->kv, cv.lp, cv.wps)) {
    plan->kv.lp = cv.lp;
    plan->kv.wps = cv.wps;
    choice_from_kv(plan->tune, plan->kv, plan->info.n);
    plan->tune.cached = 1;
    return HP_OK;
  }
  int rc;
  if ((rc = plan_variant(plan, 0))) return rc;
  const Kv def = plan->kv;
  // sample: a few resident rounds of the widest variant
  const int64_t sample = std::min<int64_t>(plan->info.paths, (int64_t)ctx->cus * 4 * 64 * 2);
  DevBuf e, st;
  if ((rc = e.alloc((size_t)sample * plan->info.n * sizeof(hp_c64)))) return rc;
  if ((rc = st.alloc((size_t)sample * sizeof(int32_t)))) return rc;
  std::vector<int> codes = kv_candidates(plan->info.n, plan->P.emax, ctx->max_lds);
  if (plan_spec_eligible(plan)) codes.insert(codes.begin(), 300 + plan->info.n);
  if (!plan->P.general)
    if (const int dc = dense_code_for(plan->P)) codes.push_back(dc);
  std::vector<Kv> cands;
  for (int code : codes) {
    Kv k;
    if (!kv_decode(code, k) || check_lds(ctx, kv_lds(k, plan->P)) != HP_OK) continue;
    if (k.lanes && plan->P.general) continue;
    if (k.dense && !dense_fits(k, plan->P)) continue;
    if (k.spec && (rc = spec_prepare(plan, k))) return rc;
    for (const Kv &v : tune_shapes(ctx, k, plan->P)) cands.push_back(v);
  }
  DevSys d = plan->P.sys[0];
  d.n_paths = sample;
  d.ids = nullptr;
  HIP_TRY(hipMemcpyAsync(plan->dev.sys.p, &d, sizeof(d), hipMemcpyHostToDevice, ctx->stream));
  Kv best_k = def;
  rc = tune_pick(cands, def, [&](const Kv &k, float &ms) {
    int r = launch_persistent(ctx, plan->dev, plan->P, k, plan->tol, sample, e.as<hp_c64>(),
                              st.as<int32_t>(), nullptr, ctx->stream, nullptr, nullptr, nullptr,
                              nullptr, -1, &plan->eg);
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    return HP_OK;
  }, best_k, plan->tune);
  if (rc) return rc;
  plan->kv = best_k;
  choice_from_kv(plan->tune, best_k, plan->info.n);
  tune_store(key, TuneVal{best_k.code, best_k.lp, best_k.wps});
  return HP_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// A plan for f; with g and/or start given, a general start system and
// explicit start points (n_start of them, host memory, [n_start][n]).
int plan_create(hp_context *ctx, const hp_system *f, const hp_system *g, const hp_c64 *start,
                int64_t n_start, hp_c64 gamma, const hp_tolerances *tol, int32_t tune,
                bool spec_default, hp_plan **out) {
  if (!ctx || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  int rc = check_tol(tol);
  if (rc) return rc;
  if (!std::isfinite(gamma.re) || !std::isfinite(gamma.im) || (gamma.re == 0 && gamma.im == 0))
    return fail(HP_E_INVALID_ARG, "gamma must be finite and nonzero");
  std::unique_ptr<hp_plan> p(new hp_plan());
  p->ctx = ctx;
  p->spec_default = spec_default;
  if ((rc = check_system(f, p->info))) return rc;
  SysInfo ginfo;
  if (g) {
    if ((rc = check_system(g, ginfo))) return fail(rc, "start system g: " + g_err);
    if (g->n != f->n) return fail(HP_E_INVALID_ARG, "g and f must have the same n");
    if (!start) return fail(HP_E_INVALID_ARG, "a general start system needs its start points");
  }
  if (start) {
    if (n_start < 0) return fail(HP_E_INVALID_ARG, "n_paths < 0");
    for (int64_t i = 0; i < n_start * f->n; ++i)
      if (!std::isfinite(start[i].re) || !std::isfinite(start[i].im))
        return fail(HP_E_INVALID_ARG, "start points must be finite");
    p->info.paths = n_start;
  }
  p->n_terms = f->n_terms;
  if (tol) p->tol = *tol;
  else hp_default_tolerances(&p->tol);
  p->gamma = gamma;
  HIP_TRY(hipSetDevice(ctx->device));
  const double2 *dstart = nullptr;
  if (start) {
    if ((rc = p->start_dev.alloc((size_t)std::max<int64_t>(1, n_start) * f->n * sizeof(hp_c64))))
      return rc;
    if (n_start > 0)
      HIP_TRY(hipMemcpy(p->start_dev.p, start, (size_t)n_start * f->n * sizeof(hp_c64),
                        hipMemcpyHostToDevice));
    dstart = p->start_dev.as<double2>();
  }
  pack_append(p->P, f, p->info, gamma, p->info.paths, 0, 0, nullptr, g, g ? ginfo.emax : 0,
              dstart);
  if ((rc = p->dev.upload(p->P, ctx->stream))) return rc;
  if ((rc = plan_variant(p.get(), 0))) return rc;
  if (tune && (rc = autotune(p.get()))) return rc;
  context_adopt(ctx);
  *out = p.release();
  return HP_OK;
}

}  // namespace

extern "C" {

int hp_plan_create_general(hp_context *ctx, const hp_system *f, const hp_system *g,
                           const hp_c64 *start, int64_t n_start, hp_c64 gamma,
                           const hp_tolerances *tol, int32_t tune, hp_plan **out) {
  if (!start) return fail(HP_E_INVALID_ARG, "a general plan needs its start points");
  return plan_create(ctx, f, g, start, n_start, gamma, tol, tune, true, out);
}

int hp_plan_create(hp_context *ctx, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
                   int32_t tune, hp_plan **out) {
  return plan_create(ctx, f, nullptr, nullptr, 0, gamma, tol, tune, true, out);
}

void hp_plan_destroy(hp_plan *plan) {
  if (!plan) return;
  hp_context *ctx = plan->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  delete plan;
  context_orphan(ctx);
}

int hp_spec_compile_form(const hp_system *f, int32_t form, int64_t *code_bytes) {
  if (!code_bytes) return fail(HP_E_INVALID_ARG, "NULL argument");
  *code_bytes = 0;
  if (form < 0 || form > 2) return fail(HP_E_INVALID_ARG, "form must be 0, 1 or 2");
  SysInfo info;
  int rc = check_system(f, info);
  if (rc) return rc;
  Packed P;
  pack_append(P, f, info, hp_c64{1.0, 0.0}, info.paths, 0, 0, nullptr);
  const DevSys &d = P.sys[0];
  if (!hp::spec_eligible(f->n, P.terms.data(), d.n_terms))
    return fail(HP_E_UNSUPPORTED_N, "system too large for a specialised kernel");
  std::vector<char> code;
  std::string log;
  rc = hp::spec_compile(hp::spec_source(f->n, d.deg, P.terms.data(), d.n_terms, form == 1, form == 2),
                        code, log);
  if (rc) return fail(HP_E_DEVICE, "specialised kernel (form " + std::to_string(form) + "): " + log);
  *code_bytes = (int64_t)code.size();
  return HP_OK;
}

int hp_spec_compile(const hp_system *f, int64_t *code_bytes) {
  if (!code_bytes) return fail(HP_E_INVALID_ARG, "NULL argument");
  int64_t serving = 0;
  int rc = hp_spec_compile_form(f, 0, code_bytes);
  if (rc == HP_OK) rc = hp_spec_compile_form(f, 1, &serving);
  return rc;
}

int hp_plan_set_variant(hp_plan *plan, int32_t variant) {
  if (!plan) return fail(HP_E_INVALID_ARG, "plan is NULL");
  return plan_variant(plan, variant);
}

int hp_plan_set_launch(hp_plan *plan, int32_t paths_per_wave, int32_t waves_per_simd) {
  if (!plan) return fail(HP_E_INVALID_ARG, "plan is NULL");
  if (!shape_ok(plan->kv, paths_per_wave, waves_per_simd))
    return fail(HP_E_INVALID_ARG, "paths_per_wave must be 0 (or 1..64 on a specialised or dense "
                                  "kernel), waves_per_simd 0..64");
  plan->kv.lp = paths_per_wave == hp::kLanes ? 0 : paths_per_wave;
  plan->kv.wps = waves_per_simd;
  return HP_OK;
}

int hp_plan_tuning(const hp_plan *plan, hp_tune_choice *out) {
  if (!plan || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  *out = plan->tune;
  return HP_OK;
}

int hp_plan_track_device(hp_plan *plan, const int64_t *ids, int64_t n_paths, hp_c64 *endpoints,
                         int32_t *status, hp_path_stats *stats, int32_t mode, void *stream) {
  if (!plan) return fail(HP_E_INVALID_ARG, "plan is NULL");
  if (n_paths < 0) return fail(HP_E_INVALID_ARG, "n_paths < 0");
  if (!ids && n_paths > plan->info.paths)
    return fail(HP_E_INVALID_ARG, "n_paths exceeds the number of total-degree paths");
  if (n_paths > 0 && (!endpoints || !status)) return fail(HP_E_INVALID_ARG, "NULL output");
  if (mode != HP_PLAIN && mode != HP_BATCHED) return fail(HP_E_INVALID_ARG, "unknown mode");
  hp_context *ctx = plan->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  const double t0 = now_ms();
  ctx->last = hp_timing{};
  timing_shape(ctx->last, plan->kv, plan->info.n);
  if (n_paths == 0) return HP_OK;
  int rc;
  if (mode == HP_PLAIN) {
    if ((rc = track_plain(plan, ids, n_paths, endpoints, status, stats, s))) return rc;
  } else {
    DevSys d = plan->P.sys[0];
    d.n_paths = n_paths;
    d.ids = ids;
    HIP_TRY(hipMemcpyAsync(plan->dev.sys.p, &d, sizeof(d), hipMemcpyHostToDevice, s));
    int groups = 0;
    if ((rc = launch_persistent(ctx, plan->dev, plan->P, plan->kv, plan->tol, n_paths,
                                endpoints, status, stats, s, &groups, nullptr, nullptr, nullptr,
                                -1, &plan->eg)))
      return rc;
    ctx->last.launches = 1;
    ctx->last.groups = groups;
  }
  HIP_TRY(hipEventSynchronize(ctx->ev1));
  float ms = 0.f, eg = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->evm));
  HIP_TRY(hipEventElapsedTime(&eg, ctx->evm, ctx->ev1));
  ctx->last.kernel_ms = ms;
  ctx->last.endgame_ms = eg;
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

int hp_track_paths(hp_context *ctx, const hp_system *f, const hp_system *g, const hp_c64 *start,
                   int64_t n_paths, hp_c64 gamma, const hp_tolerances *tol, hp_c64 *endpoints,
                   int32_t *status, hp_path_stats *stats, int32_t mode) {
  if (!ctx) return fail(HP_E_INVALID_ARG, "context is NULL");
  if (g && !start) return fail(HP_E_INVALID_ARG, "a general start system needs its start points");
  if (n_paths < 0 || (n_paths > 0 && (!endpoints || !status)))
    return fail(HP_E_INVALID_ARG, "bad outputs");
  const double t0 = now_ms();
  hp_plan *plan = nullptr;
  int rc = plan_create(ctx, f, g, start, n_paths, gamma, tol, 0, false, &plan);
  if (rc) return rc;
  std::unique_ptr<hp_plan, void (*)(hp_plan *)> guard(plan, hp_plan_destroy);
  if (n_paths > plan->info.paths)
    return fail(HP_E_INVALID_ARG, "n_paths exceeds the number of total-degree paths");
  const int n = plan->info.n;
  DevBuf e, st, sts;
  if ((rc = e.alloc((size_t)std::max<int64_t>(1, n_paths) * n * sizeof(hp_c64)))) return rc;
  if ((rc = st.alloc((size_t)std::max<int64_t>(1, n_paths) * sizeof(int32_t)))) return rc;
  if (stats && (rc = sts.alloc((size_t)std::max<int64_t>(1, n_paths) * sizeof(hp_path_stats))))
    return rc;
  rc = hp_plan_track_device(plan, nullptr, n_paths, e.as<hp_c64>(), st.as<int32_t>(),
                            stats ? sts.as<hp_path_stats>() : nullptr, mode, nullptr);
  if (rc) return rc;
  if (n_paths > 0) {
    HIP_TRY(hipMemcpy(endpoints, e.p, (size_t)n_paths * n * sizeof(hp_c64), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(status, st.p, (size_t)n_paths * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (stats)
      HIP_TRY(hipMemcpy(stats, sts.p, (size_t)n_paths * sizeof(hp_path_stats), hipMemcpyDeviceToHost));
  }
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

void hp_default_tolerances_dd(hp_tolerances *t) {
  if (!t) return;
  hp_default_tolerances(t);
  t->tol_final = 1e-26;
}

int hp_track_paths_dd(hp_context *ctx, const hp_system *f, const hp_c64 *start, int64_t n_paths,
                      hp_c64 gamma, const hp_tolerances *tol, hp_c64 *endpoints_hi,
                      hp_c64 *endpoints_lo, int32_t *status, hp_path_stats *stats) {
  if (!ctx) return fail(HP_E_INVALID_ARG, "context is NULL");
  if (n_paths < 0 || (n_paths > 0 && (!endpoints_hi || !endpoints_lo || !status)))
    return fail(HP_E_INVALID_ARG, "bad outputs");
  int rc = check_tol(tol);
  if (rc) return rc;
  if (!std::isfinite(gamma.re) || !std::isfinite(gamma.im) || (gamma.re == 0 && gamma.im == 0))
    return fail(HP_E_INVALID_ARG, "gamma must be finite and nonzero");
  SysInfo info;
  if ((rc = check_system(f, info))) return rc;
  const int n = f->n;
  if (!start && n_paths > info.paths)
    return fail(HP_E_INVALID_ARG, "n_paths exceeds the number of total-degree paths");
  if (start)
    for (int64_t i = 0; i < n_paths * n; ++i)
      if (!std::isfinite(start[i].re) || !std::isfinite(start[i].im))
        return fail(HP_E_INVALID_ARG, "start points must be finite");
  hp_tolerances T;
  if (tol) T = *tol;
  else hp_default_tolerances_dd(&T);
  const double t0 = now_ms();
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->last = hp_timing{};
  if (n_paths == 0) return HP_OK;
  DevBuf dstart;
  if (start) {
    if ((rc = dstart.alloc((size_t)n_paths * n * sizeof(hp_c64)))) return rc;
    HIP_TRY(hipMemcpy(dstart.p, start, (size_t)n_paths * n * sizeof(hp_c64), hipMemcpyHostToDevice));
  }
  Packed P;
  pack_append(P, f, info, gamma, n_paths, 0, 0, nullptr, nullptr, 0,
              start ? dstart.as<double2>() : nullptr);
  DevTables dev;
  if ((rc = dev.upload(P, ctx->stream))) return rc;
  DevBuf e, elo, st, sts;
  if ((rc = e.alloc((size_t)n_paths * n * sizeof(hp_c64))) ||
      (rc = elo.alloc((size_t)n_paths * n * sizeof(hp_c64))) ||
      (rc = st.alloc((size_t)n_paths * sizeof(int32_t))) ||
      (stats && (rc = sts.alloc((size_t)n_paths * sizeof(hp_path_stats)))))
    return rc;
  KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.sys = dev.sys.as<DevSys>();
  a.n_systems = 1;
  a.tcoef = dev.tcoef.as<double2>();
  a.tmeta = dev.tmeta.as<uint4>();
  a.eqp = dev.kp.as<int32_t>();
  a.roots = dev.roots.as<double2>();
  a.qhead = dev.qhead.as<unsigned long long>();
  a.endpoints = e.as<double2>();
  a.endpoints_lo = elo.as<double2>();
  a.status = st.as<int32_t>();
  a.stats = stats ? sts.as<hp_path_stats>() : nullptr;
  a.tol = dev_tol(T);
  int per_cu = 0;
  HIP_TRY((hipError_t)hp_ddtrack_per_cu(n, &per_cu));
  if (per_cu < 1) return fail(HP_E_DEVICE, "double-double kernel does not fit on a compute unit");
  const int64_t per_wave = hp::kLanes / n;
  const int64_t groups = std::min<int64_t>((int64_t)ctx->cus * per_cu,
                                           std::max<int64_t>(1, (n_paths + per_wave - 1) / per_wave));
  HIP_TRY(hipMemsetAsync(dev.qhead.p, 0, sizeof(unsigned long long), ctx->stream));
  HIP_TRY(hipEventRecord(ctx->ev0, ctx->stream));
  HIP_TRY((hipError_t)hp_launch_ddtrack(n, a, (int)groups, ctx->stream));
  HIP_TRY(hipEventRecord(ctx->ev1, ctx->stream));
  HIP_TRY(hipEventSynchronize(ctx->ev1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  HIP_TRY(hipMemcpy(endpoints_hi, e.p, (size_t)n_paths * n * sizeof(hp_c64), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(endpoints_lo, elo.p, (size_t)n_paths * n * sizeof(hp_c64), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(status, st.p, (size_t)n_paths * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (stats)
    HIP_TRY(hipMemcpy(stats, sts.p, (size_t)n_paths * sizeof(hp_path_stats), hipMemcpyDeviceToHost));
  ctx->last.kernel_ms = ms;
  ctx->last.launches = 1;
  ctx->last.groups = (int32_t)groups;
  ctx->last.paths_per_wave = (int32_t)per_wave;
  ctx->last.lanes_per_path = n;
  ctx->last.max_n = n;
  ctx->last.variant = 500 + n;
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

int hp_batch_layout(const hp_system *fs, int32_t n_systems, int64_t *path_offsets,
                    int64_t *x_offsets) {
  if (!fs || n_systems < 1 || !path_offsets || !x_offsets)
    return fail(HP_E_INVALID_ARG, "bad batch arguments");
  path_offsets[0] = 0;
  x_offsets[0] = 0;
  for (int s = 0; s < n_systems; ++s) {
    SysInfo info;
    int rc = check_system(&fs[s], info);
    if (rc) return fail(rc, "system " + std::to_string(s) + ": " + g_err);
    path_offsets[s + 1] = path_offsets[s] + info.paths;
    x_offsets[s + 1] = x_offsets[s] + info.paths * info.n;
  }
  return HP_OK;
}

int hp_track_batch(hp_context *ctx, const hp_system *fs, int32_t n_systems, const hp_c64 *gammas,
                   const hp_tolerances *tol, hp_c64 *endpoints, int32_t *status,
                   hp_path_stats *stats) {
  if (!ctx || !fs || n_systems < 1 || !gammas || !endpoints || !status)
    return fail(HP_E_INVALID_ARG, "bad batch arguments");
  int rc = check_tol(tol);
  if (rc) return rc;
  hp_tolerances T;
  if (tol) T = *tol;
  else hp_default_tolerances(&T);
  const double t0 = now_ms();
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<int64_t> po(n_systems + 1), xo(n_systems + 1);
  Packed P;
  int64_t total_terms = 0;
  if ((rc = pack_batch(fs, n_systems, gammas, po, xo, P, total_terms))) return rc;
  // the tuned launch of batches of this shape, if any (hp_tune_batch)
  Kv kv = kv_pick(P);
  TuneVal cv;
  if (tune_lookup(tune_key_batch(ctx->cus, P, total_terms), cv)) {
    Kv k;
    if (batch_variant_ok(ctx, P, cv.code, k) && shape_ok(k, cv.lp, cv.wps)) {
      k.lp = cv.lp;
      k.wps = cv.wps;
      kv = k;
    }
  }
  DevTables dev;
  if ((rc = dev.upload(P, ctx->stream))) return rc;
  DevBuf e, st, sts;
  const int64_t total = po[n_systems];
  if ((rc = e.alloc((size_t)std::max<int64_t>(1, xo[n_systems]) * sizeof(hp_c64)))) return rc;
  if ((rc = st.alloc((size_t)std::max<int64_t>(1, total) * sizeof(int32_t)))) return rc;
  if (stats && (rc = sts.alloc((size_t)std::max<int64_t>(1, total) * sizeof(hp_path_stats))))
    return rc;
  int groups = 0;
  ctx->last = hp_timing{};
  EgList egl;
  if ((rc = launch_persistent(ctx, dev, P, kv, T, total, e.as<hp_c64>(),
                              st.as<int32_t>(), stats ? sts.as<hp_path_stats>() : nullptr,
                              ctx->stream, &groups, nullptr, nullptr, nullptr, -1, &egl)))
    return rc;
  HIP_TRY(hipEventSynchronize(ctx->ev1));
  float ms = 0.f, eg = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->evm));
  HIP_TRY(hipEventElapsedTime(&eg, ctx->evm, ctx->ev1));
  ctx->last.endgame_ms = eg;
  HIP_TRY(hipMemcpy(endpoints, e.p, (size_t)xo[n_systems] * sizeof(hp_c64), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(status, st.p, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (stats)
    HIP_TRY(hipMemcpy(stats, sts.p, (size_t)total * sizeof(hp_path_stats), hipMemcpyDeviceToHost));
  ctx->last.kernel_ms = ms;
  ctx->last.launches = 1;
  ctx->last.groups = groups;
  timing_shape(ctx->last, kv, P.nl);
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

int hp_tune_batch(hp_context *ctx, const hp_system *fs, int32_t n_systems, const hp_c64 *gammas,
                  const hp_tolerances *tol, hp_tune_choice *out) {
  if (!ctx || !fs || n_systems < 1 || !gammas || !out)
    return fail(HP_E_INVALID_ARG, "bad batch arguments");
  *out = hp_tune_choice{};
  int rc = check_tol(tol);
  if (rc) return rc;
  hp_tolerances T;
  if (tol) T = *tol;
  else hp_default_tolerances(&T);
  HIP_TRY(hipSetDevice(ctx->device));
  std::vector<int64_t> po(n_systems + 1), xo(n_systems + 1);
  Packed P;
  int64_t total_terms = 0;
  if ((rc = pack_batch(fs, n_systems, gammas, po, xo, P, total_terms))) return rc;
  const Kv def = kv_pick(P);
  std::vector<Kv> cands;
  std::vector<int> codes;
  if (const int dc = dense_code_for(P)) codes.push_back(dc);
  for (int v : hp::kNmaxVariants) codes.push_back(v);
  for (int code : codes) {
    Kv k;
    if (!batch_variant_ok(ctx, P, code, k)) continue;
    for (const Kv &v : tune_shapes(ctx, k, P)) cands.push_back(v);
  }
  // sample: every system's first paths, a share of about two resident rounds
  const int64_t total = po[n_systems];
  const int64_t want = std::min<int64_t>(total, (int64_t)ctx->cus * 4 * 64 * 2);
  int64_t sample = 0;
  for (DevSys &d : P.sys) {
    d.n_paths = std::max<int64_t>(1, (d.n_paths * want + total - 1) / total);
    sample += d.n_paths;
  }
  DevTables dev;
  if ((rc = dev.upload(P, ctx->stream))) return rc;
  DevBuf e, st;
  EgList eg;
  if ((rc = e.alloc((size_t)std::max<int64_t>(1, xo[n_systems]) * sizeof(hp_c64)))) return rc;
  if ((rc = st.alloc((size_t)std::max<int64_t>(1, total) * sizeof(int32_t)))) return rc;
  Kv best = def;
  rc = tune_pick(cands, def, [&](const Kv &k, float &ms) {
    int r = launch_persistent(ctx, dev, P, k, T, sample, e.as<hp_c64>(), st.as<int32_t>(), nullptr,
                              ctx->stream, nullptr, nullptr, nullptr, nullptr, -1, &eg);
    if (r) return r;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    return HP_OK;
  }, best, *out);
  if (rc) return rc;
  choice_from_kv(*out, best, P.nl);
  tune_store(tune_key_batch(ctx->cus, P, total_terms), TuneVal{best.code, best.lp, best.wps});
  return HP_OK;
}

int64_t hp_find_duplicates(int32_t n, int64_t n_paths, const hp_c64 *x, const int32_t *status,
                           double rel, int64_t *pairs, int64_t max_pairs) {
  if (n < 1 || n_paths < 0 || (n_paths > 0 && (!x || !status)))
    return fail(HP_E_INVALID_ARG, "bad arguments"), -1;
  // projection weights with sum |u_j| + |v_j| = 1, so |proj(a) - proj(b)| <= ||a - b||_inf
  std::mt19937_64 rng(0x9e3779b97f4a7c15ULL);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  std::vector<double> wr(n), wi(n);
  double sum = 0.0;
  for (int j = 0; j < n; ++j) {
    wr[j] = U(rng);
    wi[j] = U(rng);
    sum += std::fabs(wr[j]) + std::fabs(wi[j]);
  }
  for (int j = 0; j < n; ++j) {
    wr[j] /= sum;
    wi[j] /= sum;
  }
  struct Item {
    double proj, norm;
    int64_t idx;
  };
  std::vector<Item> items;
  for (int64_t p = 0; p < n_paths; ++p) {
    if (status[p] != HP_CONVERGED) continue;
    double pr = 0.0, nm = 0.0;
    for (int j = 0; j < n; ++j) {
      const hp_c64 z = x[p * n + j];
      pr += wr[j] * z.re + wi[j] * z.im;
      nm = std::max(nm, std::hypot(z.re, z.im));
    }
    items.push_back({pr, nm, p});
  }
  std::sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
    return a.proj < b.proj || (a.proj == b.proj && a.idx < b.idx);
  });
  int64_t count = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    for (size_t k = i + 1; k < items.size(); ++k) {
      const double win = rel * std::max(1.0, std::max(items[i].norm, items[k].norm));
      if (items[k].proj - items[i].proj > win) break;
      int64_t a = std::min(items[i].idx, items[k].idx), b = std::max(items[i].idx, items[k].idx);
      const double scale = std::max(1.0, a == items[i].idx ? items[i].norm : items[k].norm);
      double d = 0.0;
      for (int j = 0; j < n; ++j) {
        const hp_c64 za = x[a * n + j], zb = x[b * n + j];
        d = std::max(d, std::hypot(za.re - zb.re, za.im - zb.im));
      }
      if (d <= rel * scale) {
        if (count < max_pairs && pairs) {
          pairs[2 * count] = a;
          pairs[2 * count + 1] = b;
        }
        ++count;
      }
    }
  }
  return count;
}

}  // extern "C"

namespace {

// Projection weights of the duplicate scans (host and device): uniform in
// [-1, 1] from a fixed seed, scaled to sum |u_j| + |v_j| = 1, so that
// |proj(a) - proj(b)| <= ||a - b||_inf.
void dup_weights(int n, double *w) {
  std::mt19937_64 rng(0x9e3779b97f4a7c15ULL);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  double sum = 0.0;
  for (int j = 0; j < 2 * n; ++j) {
    w[j] = U(rng);
    sum += std::fabs(w[j]);
  }
  for (int j = 0; j < 2 * n; ++j) w[j] /= sum;
}

// The device duplicate scan into the context's workspace: *found = pairs
// found; the first min(found, max_pairs) pairs are at W.pairs (device).
// Waits for stream s (two counts read back).
int dup_scan(hp_context *ctx, int n, int64_t n_paths, const hp_c64 *e, const int32_t *st,
             double rel, int64_t want_pairs, int64_t *found, hipStream_t s) {
  DupWork &W = ctx->dup;
  int rc;
  if ((rc = W.reserve(1, want_pairs))) return rc;
  hp::DupArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.n_paths = n_paths;
  a.endpoints = (const double2 *)e;
  a.status = st;
  a.rel = rel;
  dup_weights(n, a.w);
  unsigned long long cnt[2] = {0, 0};
  for (int pass = 0; pass < 2; ++pass) {
    a.keys = W.keys.as<double>();
    a.ids = W.ids.as<long long>();
    a.keys_sorted = W.keys_sorted.as<double>();
    a.ids_sorted = W.ids_sorted.as<long long>();
    a.cap = W.cap;
    a.count = W.counts.as<unsigned long long>();
    a.pair_count = a.count + 1;
    a.temp = W.temp.p;
    a.temp_bytes = W.temp_bytes;
    HIP_TRY(hipMemsetAsync(W.counts.p, 0, 2 * sizeof(unsigned long long), s));
    HIP_TRY((hipError_t)hp_launch_dup_project(a, s));
    HIP_TRY(hipMemcpyAsync(cnt, W.counts.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((long long)cnt[0] <= W.cap) break;
    if ((rc = W.reserve((long long)cnt[0], want_pairs))) return rc;  // more converged paths than room
  }
  const long long m = (long long)cnt[0];
  a.pairs = W.pairs.as<long long>();
  a.max_pairs = W.max_pairs;
  HIP_TRY((hipError_t)hp_launch_dup_sort(a, m, s));
  HIP_TRY((hipError_t)hp_launch_dup_scan(a, m, s));
  HIP_TRY(hipMemcpyAsync(&cnt[1], a.pair_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *found = (int64_t)cnt[1];
  return HP_OK;
}

}  // namespace

extern "C" {

int hp_find_duplicates_device(hp_context *ctx, int32_t n, int64_t n_paths, const hp_c64 *endpoints,
                              const int32_t *status, double rel, int64_t *pairs, int64_t max_pairs,
                              int64_t *n_pairs, void *stream) {
  if (!ctx || !n_pairs) return fail(HP_E_INVALID_ARG, "NULL argument");
  if (n < 1 || n > HP_MAX_N || n_paths < 0 || max_pairs < 0 || !(rel >= 0.0) ||
      (n_paths > 0 && (!endpoints || !status)) || (max_pairs > 0 && !pairs))
    return fail(HP_E_INVALID_ARG, "bad arguments");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  int64_t found = 0;
  int rc = dup_scan(ctx, n, n_paths, endpoints, status, rel, max_pairs, &found, s);
  if (rc) return rc;
  const int64_t k = std::min(found, max_pairs);
  if (k > 0)
    HIP_TRY(hipMemcpyAsync(pairs, ctx->dup.pairs.p, (size_t)k * 2 * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, s));
  *n_pairs = found;
  return HP_OK;
}

int hp_find_duplicates_device_static(hp_context *ctx, int32_t n, int64_t n_paths,
                                     const hp_c64 *endpoints, const int32_t *status, double rel,
                                     int64_t *pairs, int64_t max_pairs, int64_t *n_pairs,
                                     void *stream) {
  if (!ctx || !n_pairs) return fail(HP_E_INVALID_ARG, "NULL argument");
  if (n < 1 || n > HP_MAX_N || n_paths < 0 || max_pairs < 0 || !(rel >= 0.0) ||
      (n_paths > 0 && (!endpoints || !status)) || (max_pairs > 0 && !pairs))
    return fail(HP_E_INVALID_ARG, "bad arguments");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  hp::DupArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.n_paths = n_paths;
  a.endpoints = (const double2 *)endpoints;
  a.status = status;
  a.rel = rel;
  dup_weights(n, a.w);
  a.pairs = (long long *)pairs;
  a.max_pairs = max_pairs;
  long long found = 0;
  std::string err;
  const int rc = hp_dup_static_scan(ctx->device, a, &found, err, s);
  if (rc == -2) return fail(HP_E_BUDGET, err);
  if (rc) return fail(HP_E_DEVICE, "static duplicate scan: " + err);
  *n_pairs = found;
  return HP_OK;
}

int hp_plan_solve_device(hp_plan *plan, hp_c64 *endpoints, int32_t *status, hp_path_stats *stats,
                         int64_t *pairs_found, int64_t *pairs_left, void *stream) {
  if (!plan || !endpoints || !status) return fail(HP_E_INVALID_ARG, "NULL argument");
  if (plan->P.general) return fail(HP_E_INVALID_ARG, "a solve tracks the total-degree start system");
  hp_context *ctx = plan->ctx;
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  const double t0 = now_ms();
  const int n = plan->info.n;
  const int64_t P = plan->info.paths;
  int rc = hp_plan_track_device(plan, nullptr, P, endpoints, status, stats, HP_BATCHED, s);
  if (rc) return rc;
  const hp_timing track = ctx->last;
  const double tp = now_ms();
  constexpr double kRel = 1e-6;
  int64_t found = 0;
  if ((rc = dup_scan(ctx, n, P, endpoints, status, kRel, 1 << 16, &found, s))) return rc;
  if (found > ctx->dup.max_pairs &&
      (rc = dup_scan(ctx, n, P, endpoints, status, kRel, found, &found, s)))
    return rc;
  int64_t left = found;
  if (found > 0) {
    // both paths of every pair, each once, tracked again with tighter steps
    std::vector<int64_t> pr(2 * found);
    HIP_TRY(hipMemcpy(pr.data(), ctx->dup.pairs.p, pr.size() * sizeof(int64_t),
                      hipMemcpyDeviceToHost));
    std::sort(pr.begin(), pr.end());
    pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
    const int64_t m = (int64_t)pr.size();
    DevBuf dids, e2, st2, sts2;
    if ((rc = dids.alloc(m * sizeof(int64_t))) || (rc = e2.alloc((size_t)m * n * sizeof(hp_c64))) ||
        (rc = st2.alloc((size_t)m * sizeof(int32_t))) ||
        (rc = sts2.alloc((size_t)m * sizeof(hp_path_stats))))
      return rc;
    HIP_TRY(hipMemcpyAsync(dids.p, pr.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
    const hp_tolerances keep = plan->tol;
    plan->tol.h_max = std::min(keep.h_max, 0.01);
    plan->tol.tol_corr = std::min(keep.tol_corr, 1e-10);
    rc = hp_plan_track_device(plan, dids.as<int64_t>(), m, e2.as<hp_c64>(), st2.as<int32_t>(),
                              sts2.as<hp_path_stats>(), HP_BATCHED, s);
    plan->tol = keep;
    if (rc) return rc;
    HIP_TRY((hipError_t)hp_launch_scatter(dids.as<long long>(), m, n, e2.as<double2>(),
                                          st2.as<int32_t>(), sts2.as<hp_path_stats>(),
                                          (double2 *)endpoints, status, stats, s));
    if ((rc = dup_scan(ctx, n, P, endpoints, status, kRel, 0, &left, s))) return rc;
  }
  if (pairs_found) *pairs_found = found;
  if (pairs_left) *pairs_left = left;
  ctx->last = track;
  ctx->last.post_ms = now_ms() - tp;
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

int hp_solve(hp_context *ctx, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
             hp_c64 *endpoints, int32_t *status, hp_path_stats *stats, int64_t *remaining_pairs) {
  if (!ctx || !endpoints || !status) return fail(HP_E_INVALID_ARG, "NULL argument");
  const double t0 = now_ms();
  hp_plan *plan = nullptr;
  int rc = hp_plan_create(ctx, f, gamma, tol, 0, &plan);
  if (rc) return rc;
  std::unique_ptr<hp_plan, void (*)(hp_plan *)> guard(plan, hp_plan_destroy);
  const int n = plan->info.n;
  const int64_t P = plan->info.paths;
  DevBuf e, st, sts;
  if ((rc = e.alloc((size_t)P * n * sizeof(hp_c64)))) return rc;
  if ((rc = st.alloc((size_t)P * sizeof(int32_t)))) return rc;
  if ((rc = sts.alloc((size_t)P * sizeof(hp_path_stats)))) return rc;
  int64_t left = 0;
  rc = hp_plan_solve_device(plan, e.as<hp_c64>(), st.as<int32_t>(), sts.as<hp_path_stats>(),
                            nullptr, &left, nullptr);
  if (rc) return rc;
  const hp_timing keep = ctx->last;
  HIP_TRY(hipMemcpy(endpoints, e.p, (size_t)P * n * sizeof(hp_c64), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(status, st.p, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (stats)
    HIP_TRY(hipMemcpy(stats, sts.p, (size_t)P * sizeof(hp_path_stats), hipMemcpyDeviceToHost));
  if (remaining_pairs) *remaining_pairs = left;
  ctx->last = keep;
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Homotopy membership test (Section 4.1, Example 4.1)
// ---------------------------------------------------------------------------

namespace {

// e with the constant term of each of its last n_hyper equations replaced so
// that the equation vanishes at y (a hyperplane without a constant term gets
// one).  The arrays of the result live in the given vectors.
int moved_system(const hp_system *e, int n_hyper, const hp_c64 *y, std::vector<int32_t> &eq_ptr,
                 std::vector<hp_c64> &coeff, std::vector<uint8_t> &exps, hp_system &out) {
  const int n = e->n;
  eq_ptr.assign(1, 0);
  coeff.clear();
  exps.clear();
  for (int i = 0; i < n; ++i) {
    const bool hyper = i >= n - n_hyper;
    double rre = 0.0, rim = 0.0;  // the non-constant terms at y
    int const_at = -1;
    for (int t = e->eq_ptr[i]; t < e->eq_ptr[i + 1]; ++t) {
      int deg = 0, var = -1;
      for (int j = 0; j < n; ++j) {
        const int a = e->exps[(size_t)t * n + j];
        deg += a;
        if (a) var = j;
      }
      if (hyper && deg > 1) return fail(HP_E_INVALID_ARG, "a hyperplane equation is not linear");
      if (hyper && deg == 1) {
        const hp_c64 c = e->coeff[t], v = y[var];
        rre += c.re * v.re - c.im * v.im;
        rim += c.re * v.im + c.im * v.re;
      }
      if (hyper && deg == 0 && const_at < 0) const_at = (int)coeff.size();
      coeff.push_back(e->coeff[t]);
      exps.insert(exps.end(), e->exps + (size_t)t * n, e->exps + (size_t)(t + 1) * n);
    }
    if (hyper) {
      if (const_at < 0) {
        const_at = (int)coeff.size();
        coeff.push_back(hp_c64{0.0, 0.0});
        exps.insert(exps.end(), (size_t)n, (uint8_t)0);
      }
      coeff[const_at] = hp_c64{-rre, -rim};
    }
    eq_ptr.push_back((int32_t)coeff.size());
  }
  out = hp_system{n, (int32_t)coeff.size(), eq_ptr.data(), coeff.data(), exps.data()};
  return HP_OK;
}

}  // namespace

extern "C" {

int hp_membership_test(hp_context *ctx, const hp_system *e, int32_t n_hyper, const hp_c64 *witness,
                       int64_t m, const hp_c64 *tests, int32_t n_tests, const hp_tolerances *tol,
                       double rel, hp_c64 *endpoints, int32_t *status, int32_t *member) {
  if (!ctx || !e || !witness || !tests || !endpoints || !status || !member)
    return fail(HP_E_INVALID_ARG, "NULL argument");
  SysInfo info;
  int rc = check_system(e, info);
  if (rc) return rc;
  if (n_hyper < 1 || n_hyper >= e->n || m < 1 || n_tests < 1 || !(rel >= 0.0))
    return fail(HP_E_INVALID_ARG, "bad membership-test sizes");
  if ((rc = check_tol(tol))) return rc;
  hp_tolerances T;
  if (tol) T = *tol;
  else hp_default_tolerances(&T);
  const int n = e->n;
  for (int64_t k = 0; k < m * n; ++k)
    if (!std::isfinite(witness[k].re) || !std::isfinite(witness[k].im))
      return fail(HP_E_INVALID_ARG, "witness points must be finite");
  const double t0 = now_ms();
  HIP_TRY(hipSetDevice(ctx->device));
  DevBuf dstart;
  if ((rc = dstart.alloc((size_t)m * n * sizeof(hp_c64)))) return rc;
  HIP_TRY(hipMemcpy(dstart.p, witness, (size_t)m * n * sizeof(hp_c64), hipMemcpyHostToDevice));
  // one target system per test point, all with start system e and the
  // witness points as start solutions, in one launch (gamma = 1)
  Packed P;
  std::vector<std::vector<int32_t>> ep(n_tests);
  std::vector<std::vector<hp_c64>> cf(n_tests);
  std::vector<std::vector<uint8_t>> ex(n_tests);
  for (int k = 0; k < n_tests; ++k) {
    hp_system f;
    if ((rc = moved_system(e, n_hyper, tests + (size_t)k * n, ep[k], cf[k], ex[k], f))) return rc;
    SysInfo fi;
    if ((rc = check_system(&f, fi))) return rc;
    pack_append(P, &f, fi, hp_c64{1.0, 0.0}, m, (int64_t)k * m, (int64_t)k * m * n, nullptr, e,
                info.emax, dstart.as<double2>());
  }
  DevTables dev;
  if ((rc = dev.upload(P, ctx->stream))) return rc;
  const int64_t total = (int64_t)n_tests * m;
  DevBuf de, ds;
  if ((rc = de.alloc((size_t)total * n * sizeof(hp_c64))) ||
      (rc = ds.alloc((size_t)total * sizeof(int32_t))))
    return rc;
  Kv kv;
  kv_decode(nmax_for(n), kv);  // general start systems run on the group kernels
  int groups = 0;
  ctx->last = hp_timing{};
  EgList egl;
  if ((rc = launch_persistent(ctx, dev, P, kv, T, total, de.as<hp_c64>(), ds.as<int32_t>(), nullptr,
                              ctx->stream, &groups, nullptr, nullptr, nullptr, -1, &egl)))
    return rc;
  HIP_TRY(hipEventSynchronize(ctx->ev1));
  float ms = 0.f, eg = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->evm));
  HIP_TRY(hipEventElapsedTime(&eg, ctx->evm, ctx->ev1));
  HIP_TRY(hipMemcpy(endpoints, de.p, (size_t)total * n * sizeof(hp_c64), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(status, ds.p, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int k = 0; k < n_tests; ++k) {
    const hp_c64 *y = tests + (size_t)k * n;
    double ny = 0.0;
    for (int j = 0; j < n; ++j) ny = std::max(ny, std::hypot(y[j].re, y[j].im));
    member[k] = 0;
    for (int64_t p = 0; p < m; ++p) {
      const int64_t q = (int64_t)k * m + p;
      if (status[q] != HP_CONVERGED) continue;
      double d = 0.0;
      for (int j = 0; j < n; ++j)
        d = std::max(d, std::hypot(endpoints[q * n + j].re - y[j].re, endpoints[q * n + j].im - y[j].im));
      if (d <= rel * std::max(1.0, ny)) member[k] = 1;
    }
  }
  ctx->last.kernel_ms = ms;
  ctx->last.endgame_ms = eg;
  ctx->last.launches = 1;
  ctx->last.groups = groups;
  timing_shape(ctx->last, kv, n);
  ctx->last.total_ms = now_ms() - t0;
  return HP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Cascade of homotopies (Section 3.1, Example 3.1, Figure 3)
// ---------------------------------------------------------------------------

namespace {

// A system that owns its arrays.
struct OwnedSystem {
  std::vector<int32_t> eq_ptr;
  std::vector<hp_c64> coeff;
  std::vector<uint8_t> exps;
  hp_system sys{};
  void copy_from(const hp_system *s) {
    const int n = s->n;
    eq_ptr.assign(s->eq_ptr, s->eq_ptr + n + 1);
    coeff.assign(s->coeff, s->coeff + s->n_terms);
    exps.assign(s->exps, s->exps + (size_t)s->n_terms * n);
    sys = hp_system{n, s->n_terms, eq_ptr.data(), coeff.data(), exps.data()};
  }
};

// The cascade stage's target: in cur (n unknowns, the last k slack), the
// terms in z_d (unknown n - k + d - 1) leave the first n - k equations and
// equation n - k + d - 1 becomes z_d = 0.
void stage_system(const hp_system *cur, int k, int d, OwnedSystem &out) {
  const int n = cur->n, nx = n - k, zi = nx + d - 1;
  out.eq_ptr.assign(1, 0);
  out.coeff.clear();
  out.exps.clear();
  for (int i = 0; i < n; ++i) {
    if (i == zi) {
      out.coeff.push_back(hp_c64{1.0, 0.0});
      for (int j = 0; j < n; ++j) out.exps.push_back(j == zi ? 1 : 0);
    } else {
      for (int t = cur->eq_ptr[i]; t < cur->eq_ptr[i + 1]; ++t) {
        if (i < nx && cur->exps[(size_t)t * n + zi] > 0) continue;
        out.coeff.push_back(cur->coeff[t]);
        out.exps.insert(out.exps.end(), cur->exps + (size_t)t * n, cur->exps + (size_t)(t + 1) * n);
      }
    }
    out.eq_ptr.push_back((int32_t)out.coeff.size());
  }
  out.sys = hp_system{n, (int32_t)out.coeff.size(), out.eq_ptr.data(), out.coeff.data(),
                      out.exps.data()};
}

}  // namespace

extern "C" {

int hp_cascade(hp_context *ctx, const hp_system *e, int32_t k, const hp_c64 *gammas,
               const hp_tolerances *tol, double slack_tol, hp_cascade_stage *stages,
               hp_c64 *witness, int32_t *witness_dim, int64_t cap, int64_t *n_witness) {
  if (!ctx || !e || !gammas || !stages || !n_witness || (cap > 0 && (!witness || !witness_dim)))
    return fail(HP_E_INVALID_ARG, "NULL argument");
  SysInfo info;
  int rc = check_system(e, info);
  if (rc) return rc;
  if (k < 1 || k >= e->n || cap < 0 || !(slack_tol >= 0.0))
    return fail(HP_E_INVALID_ARG, "bad cascade arguments");
  const int n = e->n, nx = n - k;
  for (int j = 0; j < k; ++j)  // hyperplane j is linear and holds z_j
    for (int t = e->eq_ptr[nx + j]; t < e->eq_ptr[nx + j + 1]; ++t) {
      int deg = 0;
      for (int v = 0; v < n; ++v) deg += e->exps[(size_t)t * n + v];
      if (deg > 1) return fail(HP_E_INVALID_ARG, "a hyperplane equation is not linear");
    }
  int64_t total = 0;
  auto take = [&](const std::vector<hp_c64> &x, int64_t p, int dim) {
    if (total < cap) {
      std::memcpy(witness + total * n, x.data() + p * n, n * sizeof(hp_c64));
      witness_dim[total] = dim;
    }
    ++total;
  };
  // stage 0: the top system
  std::vector<hp_c64> ends;
  std::vector<int32_t> st;
  double kms = 0.0;
  {
    hp_plan *plan = nullptr;
    if ((rc = hp_plan_create(ctx, e, gammas[0], tol, 0, &plan))) return rc;
    std::unique_ptr<hp_plan, void (*)(hp_plan *)> guard(plan, hp_plan_destroy);
    const int64_t P = plan->info.paths;
    DevBuf de, ds;
    if ((rc = de.alloc((size_t)P * n * sizeof(hp_c64))) || (rc = ds.alloc((size_t)P * sizeof(int32_t))))
      return rc;
    if ((rc = hp_plan_solve_device(plan, de.as<hp_c64>(), ds.as<int32_t>(), nullptr, nullptr,
                                   nullptr, nullptr)))
      return rc;
    kms = ctx->last.kernel_ms;
    ends.resize((size_t)P * n);
    st.resize(P);
    HIP_TRY(hipMemcpy(ends.data(), de.p, ends.size() * sizeof(hp_c64), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st.data(), ds.p, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  }
  OwnedSystem cur, nxt;
  cur.copy_from(e);
  for (int s = 0; s <= k; ++s) {
    const int d = k - s;
    hp_cascade_stage &S = stages[s];
    std::memset(&S, 0, sizeof(S));
    S.dim = d;
    S.paths = (int64_t)st.size();
    S.kernel_ms = kms;
    std::vector<hp_c64> starts;
    for (int64_t p = 0; p < (int64_t)st.size(); ++p) {
      if (st[p] != HP_CONVERGED) continue;
      ++S.converged;
      const hp_c64 z = d > 0 ? ends[p * n + nx + d - 1] : hp_c64{0.0, 0.0};
      if (std::hypot(z.re, z.im) <= slack_tol) {
        ++S.candidates;
        take(ends, p, d);
      } else {
        ++S.nonzero;
        starts.insert(starts.end(), ends.begin() + p * n, ends.begin() + (p + 1) * n);
      }
    }
    if (d == 0 || starts.empty()) {
      for (int r = s + 1; r <= k; ++r) {  // nothing left to track
        std::memset(&stages[r], 0, sizeof(hp_cascade_stage));
        stages[r].dim = k - r;
      }
      break;
    }
    stage_system(&cur.sys, k, d, nxt);
    const int64_t m = (int64_t)starts.size() / n;
    hp_plan *plan = nullptr;
    if ((rc = plan_create(ctx, &nxt.sys, &cur.sys, starts.data(), m, gammas[s + 1], tol, 0, false,
                          &plan)))
      return rc;
    std::unique_ptr<hp_plan, void (*)(hp_plan *)> guard(plan, hp_plan_destroy);
    DevBuf de, ds;
    if ((rc = de.alloc((size_t)m * n * sizeof(hp_c64))) || (rc = ds.alloc((size_t)m * sizeof(int32_t))))
      return rc;
    if ((rc = hp_plan_track_device(plan, nullptr, m, de.as<hp_c64>(), ds.as<int32_t>(), nullptr,
                                   HP_BATCHED, nullptr)))
      return rc;
    kms = ctx->last.kernel_ms;
    ends.resize((size_t)m * n);
    st.resize(m);
    HIP_TRY(hipMemcpy(ends.data(), de.p, ends.size() * sizeof(hp_c64), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st.data(), ds.p, st.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    cur.copy_from(&nxt.sys);
  }
  *n_witness = total;
  return HP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching over the persistent tracker, in time slices
// ---------------------------------------------------------------------------
//
// A worker thread owns a stream and an arena of path slots in HBM of at most
// the budget.  Requests are admitted in arrival order while their regions
// (slots of the arena, at most kEpochPaths per request) fit; a request with
// more paths than its region reuses the slots of finished paths.
// The work goes in epochs.  Every epoch packs, for the admitted requests in
// admission order until kEpochEntries entries are taken, a queue of each
// one's paths (those suspended in the previous epoch first, then paths not
// started yet, each holding a slot) into one multi-system persistent launch
// per kernel family.  On the one-path-per-lane families every wavefront
// stops after a budget of steps: its paths in flight are suspended to their
// slots (accepted point, t, h, counters) and resume from there in a later
// epoch, so an epoch's kernel time is bounded and a new request whose
// entries fit the next epoch starts within about one slice, while under
// load the oldest requests finish first.  The budget of each family is
// adapted so that its epochs take about the slice time.  After the launches a harvest kernel compacts the finished paths of
// the queues, which are copied to the requests' host results; their slots
// go back to the requests' free lists.
// Kernels specialised to a first-seen support are compiled on a thread of
// their own, off the submitting thread; the request joins the queue once its
// kernel is ready.

namespace {

constexpr int64_t kEpochPaths = 1 << 18;    // slots of a request's region at most
constexpr int64_t kEpochEntries = 1 << 19;  // queue entries of an epoch over all requests
constexpr int64_t kMinChunk = 4096;
constexpr int32_t kInitialBudget = 16;  // steps per wavefront in a family's first slice
constexpr int32_t kMinBudget = 4, kMaxBudget = 1 << 20;
constexpr double kDefaultSliceMs = 50.0;

struct Entry {
  int64_t pid, slot;  // path id, slot in the request's region
};

struct Request {
  int64_t id = 0;
  std::vector<int32_t> eq_ptr;
  std::vector<hp_c64> coeff;
  std::vector<uint8_t> exps;
  hp_system sys{};
  SysInfo info;
  hp_c64 gamma{};
  hp_tolerances tol{};
  double t_submit = 0.0, t_done = 0.0;
  // host results
  std::vector<hp_c64> ends;
  std::vector<int32_t> status;
  std::vector<hp_path_stats> stats;
  // progress
  int64_t next_path = 0;  // first path id not yet given a slot
  int64_t done_paths = 0;
  std::vector<Entry> live;          // paths holding a slot, not finished (queue order)
  std::vector<int64_t> free_slots;  // slots of the region holding no path
  // arena region
  int64_t region_paths = 0;  // capacity in paths
  int64_t region_off = -1;   // offset in paths into the arena
  bool admitted = false, done = false, failed = false;
  std::string error;
  int dense_code = 0;  // runs on this dense kernel (as it would alone), 0: not dense
  const hp::SpecModule *sm = nullptr;  // runs on the kernel specialised to its support
  std::string spec_src;                // that kernel's source, until it is compiled
  // this epoch's queue: entries qoff .. qoff + qlen - 1 of the epoch arrays,
  // the first qtaken of them from live
  int64_t qoff = 0, qlen = 0, qtaken = 0;

  // family key: (300, module) for a specialised kernel, (dense code,
  // nullptr) for a dense kernel, (0, nullptr) for the group kernels
  std::pair<int, const void *> family() const {
    return sm ? std::make_pair(300, (const void *)sm) : std::make_pair(dense_code, (const void *)nullptr);
  }
  // the group kernels run their queue to the end (no slot mapping, no suspension)
  bool sliceable() const { return sm || dense_code; }
};

}  // namespace

// A kernel family's launch state in the server: the requests packed into P
// (in order), their device tables and the end game's list.
struct FamState {
  std::vector<int64_t> req_ids;
  Packed P;
  DevTables dev;
  EgList eg;
  bool valid = false;
};

// Streams on which the kernel families of an epoch run side by side (with
// the server's own stream the process holds four hardware queues).
constexpr int kFamilyStreams = 3;

struct hp_server {
  hp_context *ctx = nullptr;
  size_t budget = 0, resident = 0, peak = 0;
  hipStream_t stream = nullptr;
  hipStream_t fam_stream[kFamilyStreams] = {};
  std::vector<std::array<hipEvent_t, 2>> fam_ev;  // per family of an epoch
  // per kernel family: its packed systems and device tables, kept while its
  // set of requests stays the same
  std::map<std::pair<int, const void *>, std::unique_ptr<FamState>> fam_state;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_compile;
  std::deque<std::shared_ptr<Request>> pending, to_compile;
  std::vector<std::shared_ptr<Request>> active;
  std::map<int64_t, std::shared_ptr<Request>> all;
  int64_t next_id = 1;
  bool stop = false;
  std::string error;
  std::thread worker, compiler;
  // slicing (under mu): slice time, fixed step budget (> 0 overrides the
  // adaptive one), adaptive budget per family
  double slice_ms = kDefaultSliceMs;
  int32_t fixed_steps = 0;
  std::map<std::pair<int, const void *>, int32_t> fam_budget;
  // counters (under mu)
  int64_t epochs = 0, carried = 0;
  double epoch_ms_sum = 0.0, epoch_ms_max = 0.0;
  // arena: paths are slots of (endpoints up to HP_MAX_N, status, stats)
  DevBuf a_ends, a_status, a_stats;
  int64_t arena_paths = 0;
  std::vector<std::pair<int64_t, int64_t>> free_list;  // (offset, length) in paths
  // epoch queues and harvest records: one block each, on the device and
  // pinned on the host (queue: ids, slots, path slots, endpoint offsets
  // (int64 each), n (int32); records: entry, status (int32 each), stats,
  // endpoints (HP_MAX_N each)), and the record count
  DevBuf q_dev, r_dev, r_count;
  HostBuf q_host, r_host;

  int64_t largest_free() const {
    int64_t m = 0;
    for (auto &f : free_list) m = std::max(m, f.second);
    return m;
  }
  int64_t alloc_region(int64_t len) {
    for (size_t i = 0; i < free_list.size(); ++i) {
      if (free_list[i].second >= len) {
        const int64_t off = free_list[i].first;
        free_list[i].first += len;
        free_list[i].second -= len;
        if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
        return off;
      }
    }
    return -1;
  }
  void free_region(int64_t off, int64_t len) {
    free_list.push_back({off, len});
    std::sort(free_list.begin(), free_list.end());
    std::vector<std::pair<int64_t, int64_t>> merged;
    for (auto &f : free_list) {
      if (!merged.empty() && merged.back().first + merged.back().second == f.first)
        merged.back().second += f.second;
      else
        merged.push_back(f);
    }
    free_list.swap(merged);
  }
};

namespace {

size_t slot_bytes() { return (size_t)HP_MAX_N * sizeof(hp_c64) + sizeof(int32_t) + sizeof(hp_path_stats); }

// Admits pending requests in arrival order while the arena has room (called
// with mu held).  A request gets a region for all of its paths (at most
// kEpochPaths) if one is free, else, when it is larger than the free room,
// a region of at least kMinChunk paths whose slots its paths reuse.
void admit(hp_server *S) {
  while (!S->pending.empty()) {
    auto &R = S->pending.front();
    int64_t want = std::min(std::min<int64_t>(R->info.paths, S->arena_paths), kEpochPaths);
    const int64_t room = S->largest_free();
    if (room < want) {
      if (room < std::min<int64_t>(want, kMinChunk)) break;
      want = room;
    }
    const int64_t off = S->alloc_region(want);
    if (off < 0) break;
    R->region_paths = want;
    R->region_off = off;
    R->free_slots.resize((size_t)want);
    for (int64_t k = 0; k < want; ++k) R->free_slots[(size_t)k] = want - 1 - k;  // pops 0, 1, ...
    R->admitted = true;
    S->resident += (size_t)want * slot_bytes();
    S->peak = std::max(S->peak, S->resident);
    S->active.push_back(R);
    S->pending.pop_front();
  }
}

int run_epoch(hp_server *S, std::vector<std::shared_ptr<Request>> &batch) {
  hp_context *ctx = S->ctx;
  double slice_ms;
  int32_t fixed_steps;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    slice_ms = S->slice_ms;
    fixed_steps = S->fixed_steps;
  }
  const bool sliced = fixed_steps > 0 || slice_ms > 0.0;
  const double t_epoch = now_ms();
  // one launch has one tolerance set: take the requests that share the
  // oldest active request's tolerances; the others wait for a later epoch
  const hp_tolerances tol = batch[0]->tol;

  // ---- queues, filled in admission order up to kEpochEntries entries (so
  // the oldest requests finish first and an epoch's host work is bounded):
  // a request's suspended and waiting paths first, then new paths ----
  const size_t qstride = (size_t)kEpochEntries;
  int rc;
  if ((rc = S->q_host.alloc(qstride * (4 * sizeof(int64_t) + sizeof(int32_t))))) return rc;
  int64_t *h_ids = (int64_t *)S->q_host.p, *h_slots = h_ids + qstride, *h_path = h_slots + qstride,
          *h_xoff = h_path + qstride;
  int32_t *h_n = (int32_t *)(h_xoff + qstride);
  std::vector<int32_t> h_owner;
  h_owner.reserve((size_t)kEpochEntries);
  int64_t E = 0;
  for (size_t i = 0; i < batch.size(); ++i) {
    Request &R = *batch[i];
    R.qoff = E;
    R.qlen = R.qtaken = 0;
    if (std::memcmp(&R.tol, &tol, sizeof(tol)) != 0 || E >= kEpochEntries) continue;
    const int64_t share = kEpochEntries - E;  // entries left for this request and the next
    const int n = R.info.n;
    auto push = [&](int64_t pid, int64_t slot) {
      h_ids[E] = pid;
      h_slots[E] = slot;
      h_path[E] = R.region_off + slot;
      h_xoff[E] = R.region_off * HP_MAX_N + slot * n;
      h_n[E] = n;
      h_owner.push_back((int32_t)i);
      ++E;
    };
    if (!R.sliceable()) {
      // group kernels: the next chunk of path ids in slots 0, 1, ...
      const int64_t c = std::min(std::min(R.info.paths - R.next_path, R.region_paths), share);
      for (int64_t k = 0; k < c; ++k) push(R.next_path + k, k);
      R.next_path += c;
    } else {
      const int64_t take = std::min<int64_t>((int64_t)R.live.size(), share);
      for (int64_t k = 0; k < take; ++k) push(R.live[(size_t)k].pid, R.live[(size_t)k].slot);
      R.live.erase(R.live.begin(), R.live.begin() + take);
      R.qtaken = take;
      while (E - R.qoff < share && R.next_path < R.info.paths && !R.free_slots.empty()) {
        push(R.next_path++, R.free_slots.back());
        R.free_slots.pop_back();
      }
    }
    R.qlen = E - R.qoff;
  }
  if (E == 0) return HP_OK;
  if (E > INT32_MAX) return fail(HP_E_INVALID_ARG, "epoch queue too long");
  // device copy of the queue block (same layout, stride qstride; the first
  // E entries of each array)
  if ((rc = S->q_dev.alloc(S->q_host.bytes))) return rc;
  for (int a = 0; a < 5; ++a) {
    const size_t off = (size_t)a * qstride * sizeof(int64_t), w = a < 4 ? sizeof(int64_t) : sizeof(int32_t);
    HIP_TRY(hipMemcpyAsync((char *)S->q_dev.p + off, (const char *)S->q_host.p + off, (size_t)E * w,
                           hipMemcpyHostToDevice, S->stream));
  }
  HIP_TRY(hipStreamSynchronize(S->stream));
  int64_t *d_ids = S->q_dev.as<int64_t>(), *d_slots = d_ids + qstride, *d_path = d_slots + qstride,
          *d_xoff = d_path + qstride;
  int32_t *d_n = (int32_t *)(d_xoff + qstride);

  // ---- one launch per kernel family, each request on the family it runs
  // on alone, so that its result does not depend on the other requests ----
  // families in the order of their first request; each family's packed
  // systems and device tables are kept from one epoch to the next and
  // only their queue fields refreshed while its set of requests is the same
  std::map<std::pair<int, const void *>, size_t> fam_of;
  std::vector<std::vector<size_t>> members;
  std::vector<int64_t> total;
  std::vector<Kv> fam_kv;
  std::vector<std::pair<int, const void *>> fam_key;
  for (size_t i = 0; i < batch.size(); ++i) {
    Request &R = *batch[i];
    if (R.qlen == 0) continue;
    const auto key = R.family();
    auto it = fam_of.find(key);
    if (it == fam_of.end()) {
      it = fam_of.emplace(key, members.size()).first;
      members.emplace_back();
      total.push_back(0);
      fam_key.push_back(key);
      Kv kv;
      if (R.sm) {
        kv_decode(300 + R.info.n, kv);
        kv.sm = R.sm;
      } else if (R.dense_code) {
        kv_decode(R.dense_code, kv);
      }
      // the launch shape tuned for the family's first system, when the
      // tuner chose this family's kernel for it (hp_plan_create with tuning)
      TuneVal cv;
      if ((R.sm || R.dense_code) && tune_lookup(tune_key(ctx->cus, R.info, R.sys.n_terms), cv) &&
          cv.code == kv.code && shape_ok(kv, cv.lp, cv.wps)) {
        kv.lp = cv.lp;
        kv.wps = cv.wps;
      }
      fam_kv.push_back(kv);  // group family: chosen from its systems below
    }
    members[it->second].push_back(i);
    total[it->second] += R.qlen;
  }
  std::vector<FamState *> fam(members.size());
  std::vector<bool> fam_fresh(members.size(), false);
  for (size_t f = 0; f < members.size(); ++f) {
    auto &slot = S->fam_state[fam_key[f]];
    if (!slot) slot.reset(new FamState());
    FamState &F = *slot;
    fam[f] = &F;
    std::vector<int64_t> ids;
    for (size_t i : members[f]) ids.push_back(batch[i]->id);
    const bool same = F.valid && ids == F.req_ids;
    if (!same) {
      F.P = Packed();
      F.req_ids = ids;
      F.valid = true;
      fam_fresh[f] = true;
    }
    for (size_t m = 0; m < members[f].size(); ++m) {
      Request &R = *batch[members[f][m]];
      // queue entries go to the request's arena region: path slots from
      // region_off, endpoint slots of n coordinates from region_off * HP_MAX_N
      if (!same)
        pack_append(F.P, &R.sys, R.info, R.gamma, R.qlen, R.region_off, R.region_off * HP_MAX_N,
                    nullptr);
      DevSys &d = F.P.sys[m];
      d.n_paths = R.qlen;
      if (R.sliceable()) {
        d.ids = d_ids + R.qoff;
        d.slots = d_slots + R.qoff;
        d.id_base = 0;
      } else {
        d.ids = nullptr;
        d.slots = nullptr;
        d.id_base = h_ids[R.qoff];
      }
    }
  }
  // step budget per family: -1 for the group kernels (no serving form), 0
  // (no limit) when slicing is off
  std::vector<int32_t> fam_steps(members.size(), 0);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t f = 0; f < members.size(); ++f) {
      if (fam_key[f].first == 0) fam_steps[f] = -1;
      if (fam_key[f].first == 0 || !sliced) continue;
      if (fixed_steps > 0) {
        fam_steps[f] = fixed_steps;
      } else {
        auto b = S->fam_budget.find(fam_key[f]);
        fam_steps[f] = b == S->fam_budget.end() ? kInitialBudget : b->second;
      }
    }
  }
  while (S->fam_ev.size() < members.size()) {
    std::array<hipEvent_t, 2> ev{};
    HIP_TRY(hipEventCreate(&ev[0]));
    HIP_TRY(hipEventCreate(&ev[1]));
    S->fam_ev.push_back(ev);
  }
  // every family's tables, queue heads and end-game lists first, while no
  // kernel runs: a copy or fill is itself a kernel, and issued behind
  // another family's persistent kernel it would wait for that kernel to end
  for (size_t f = 0; f < members.size(); ++f) {
    FamState &F = *fam[f];
    if (!fam_kv[f].spec && !fam_kv[f].dense) kv_decode(nmax_for(F.P.nl), fam_kv[f]);  // group kernels
    if ((rc = fam_fresh[f] ? F.dev.upload(F.P, S->stream) : F.dev.upload_sys(F.P, S->stream, true)))
      return rc;
    HIP_TRY(hipMemsetAsync(F.dev.qhead.p, 0, F.P.sys.size() * sizeof(unsigned long long), S->stream));
    if ((rc = eg_prepare(F.eg, F.dev, F.P, total[f], S->stream))) return rc;
  }
  HIP_TRY(hipStreamSynchronize(S->stream));
  // then the families run side by side (their requests' arena regions are
  // disjoint), each on one of the family streams
  for (size_t f = 0; f < members.size() && rc == HP_OK; ++f) {
    const hipStream_t fs = S->fam_stream[f % kFamilyStreams];
    FamState &F = *fam[f];
    rc = launch_persistent(ctx, F.dev, F.P, fam_kv[f], tol, total[f], S->a_ends.as<hp_c64>(),
                           S->a_status.as<int32_t>(), S->a_stats.as<hp_path_stats>(), fs, nullptr,
                           S->fam_ev[f][0], S->fam_ev[f][1], nullptr, fam_steps[f], &F.eg, true);
  }
  // every launched family ends before the harvest reads the arena
  for (int q = 0; q < kFamilyStreams; ++q) HIP_TRY(hipStreamSynchronize(S->fam_stream[q]));
  if (rc) return rc;
  std::vector<float> fam_ms(members.size(), 0.0f);
  for (size_t f = 0; f < members.size(); ++f)
    HIP_TRY(hipEventElapsedTime(&fam_ms[f], S->fam_ev[f][0], S->fam_ev[f][1]));

  // ---- harvest: finished paths to the host results, slots freed ----
  const size_t rstride = (size_t)E;
  const size_t rbytes = rstride * (2 * sizeof(int32_t) + sizeof(hp_path_stats) + HP_MAX_N * sizeof(hp_c64));
  if ((rc = S->r_dev.alloc(rbytes))) return rc;
  if ((rc = S->r_host.alloc(rbytes))) return rc;
  if ((rc = S->r_count.alloc(sizeof(unsigned)))) return rc;
  // record block: x first (16-byte aligned), then stats, entry, status
  hp_c64 *dr_x = S->r_dev.as<hp_c64>();
  hp_path_stats *dr_stats = (hp_path_stats *)(dr_x + rstride * HP_MAX_N);
  int32_t *dr_entry = (int32_t *)(dr_stats + rstride), *dr_status = dr_entry + rstride;
  hp_c64 *hr_x = (hp_c64 *)S->r_host.p;
  hp_path_stats *hr_stats = (hp_path_stats *)(hr_x + rstride * HP_MAX_N);
  int32_t *hr_entry = (int32_t *)(hr_stats + rstride), *hr_status = hr_entry + rstride;
  HIP_TRY(hipMemsetAsync(S->r_count.p, 0, sizeof(unsigned), S->stream));
  hp::CollectArgs ca;
  ca.m = E;
  ca.path_slot = (const long long *)d_path;
  ca.x_off = (const long long *)d_xoff;
  ca.n = d_n;
  ca.status = S->a_status.as<int32_t>();
  ca.endpoints = (const double2 *)S->a_ends.as<hp_c64>();
  ca.stats = S->a_stats.as<hp_path_stats>();
  ca.rec_entry = dr_entry;
  ca.rec_status = dr_status;
  ca.rec_x = (double2 *)dr_x;
  ca.rec_stats = dr_stats;
  ca.count = S->r_count.as<unsigned>();
  HIP_TRY((hipError_t)hp_launch_collect(ca, S->stream));
  unsigned cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, S->r_count.p, sizeof(unsigned), hipMemcpyDeviceToHost, S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  if ((int64_t)cnt > E) return fail(HP_E_DEVICE, "harvest count out of range");
  if (cnt) {
    HIP_TRY(hipMemcpyAsync(hr_entry, dr_entry, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipMemcpyAsync(hr_status, dr_status, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipMemcpyAsync(hr_x, dr_x, (size_t)cnt * HP_MAX_N * sizeof(hp_c64), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipMemcpyAsync(hr_stats, dr_stats, cnt * sizeof(hp_path_stats), hipMemcpyDeviceToHost, S->stream));
    HIP_TRY(hipStreamSynchronize(S->stream));
  }
  std::vector<uint8_t> finished((size_t)E, 0);
  for (unsigned r = 0; r < cnt; ++r) {
    const int64_t k = hr_entry[r];
    if (k < 0 || k >= E || finished[(size_t)k]) return fail(HP_E_DEVICE, "harvest record out of range");
    finished[(size_t)k] = 1;
    Request &R = *batch[(size_t)h_owner[(size_t)k]];
    const int64_t pid = h_ids[k], n = R.info.n;
    std::memcpy(R.ends.data() + pid * n, hr_x + (size_t)r * HP_MAX_N, (size_t)n * sizeof(hp_c64));
    R.status[(size_t)pid] = hr_status[r];
    R.stats[(size_t)pid] = hr_stats[r];
    R.done_paths += 1;
    if (R.sliceable()) R.free_slots.push_back(h_slots[k]);
  }
  // unfinished queue entries keep their slots and go first next epoch
  int64_t carried = 0;
  std::vector<bool> fam_open(members.size(), false);
  for (size_t i = 0; i < batch.size(); ++i) {
    Request &R = *batch[i];
    if (R.qlen == 0) continue;
    std::vector<Entry> keep;
    for (int64_t k = R.qoff; k < R.qoff + R.qlen; ++k)
      if (!finished[(size_t)k]) keep.push_back({h_ids[k], h_slots[k]});
    if (!keep.empty() && !R.sliceable()) return fail(HP_E_DEVICE, "a group-kernel path did not finish");
    carried += (int64_t)keep.size();
    if (!keep.empty()) fam_open[fam_of[R.family()]] = true;
    keep.insert(keep.end(), R.live.begin(), R.live.end());
    R.live.swap(keep);
  }
  const double ms = now_ms() - t_epoch;
  std::lock_guard<std::mutex> lk(S->mu);
  S->epochs += 1;
  S->carried += carried;
  S->epoch_ms_sum += ms;
  S->epoch_ms_max = std::max(S->epoch_ms_max, ms);
  // adapt each sliced family's step budget toward the slice time
  if (fixed_steps <= 0 && slice_ms > 0.0) {
    for (size_t f = 0; f < members.size(); ++f) {
      if (fam_steps[f] <= 0) continue;
      int32_t b = fam_steps[f];
      const double km = std::max(0.01, (double)fam_ms[f]);
      if (km > 1.25 * slice_ms) b = std::max(kMinBudget, (int32_t)(b * (slice_ms / km)));
      else if (km < 0.5 * slice_ms && fam_open[f]) b = std::min<int64_t>(kMaxBudget, 2 * (int64_t)b);
      S->fam_budget[fam_key[f]] = b;
    }
  }
  return HP_OK;
}

void worker_main(hp_server *S) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    std::vector<std::shared_ptr<Request>> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->active.empty(); });
      if (S->stop) {
        // requests still queued, compiling or running end as failed, so waiters return
        for (auto &R : S->pending) R->done = R->failed = true;
        for (auto &R : S->to_compile) R->done = R->failed = true;
        for (auto &R : S->active) R->done = R->failed = true;
        S->error = "server destroyed before the request finished";
        S->cv_done.notify_all();
        return;
      }
      admit(S);
      batch = S->active;
    }
    if (batch.empty()) continue;
    const int rc = run_epoch(S, batch);
    const double now = now_ms();
    std::lock_guard<std::mutex> lk(S->mu);
    std::vector<std::shared_ptr<Request>> keep;
    for (auto &R : S->active) {
      if (rc != HP_OK) {
        R->failed = true;
        R->error = g_err;
      }
      if (rc != HP_OK || R->done_paths >= R->info.paths) {
        R->done = true;
        R->t_done = now;
        // a freed region's slots hold no path: status kUnstarted throughout
        // (the harvest marks the slots of finished paths; this covers a
        // failed epoch)
        (void)hp_launch_fill_i32(S->a_status.as<int32_t>() + R->region_off, R->region_paths,
                                 hp::kUnstarted, S->stream);
        (void)hipStreamSynchronize(S->stream);
        S->resident -= (size_t)R->region_paths * slot_bytes();
        S->free_region(R->region_off, R->region_paths);
        R->live.clear();
        R->free_slots.clear();
        R->free_slots.shrink_to_fit();
      } else {
        keep.push_back(R);
      }
    }
    S->active.swap(keep);
    S->cv_done.notify_all();
  }
}

// Compiles the kernels specialised to first-seen supports, one request at a
// time; a request joins the pending queue when its kernel is loaded.
void compiler_main(hp_server *S) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    std::shared_ptr<Request> R;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_compile.wait(lk, [&] { return S->stop || !S->to_compile.empty(); });
      if (S->stop) return;
      R = S->to_compile.front();
    }
    std::string log;
    const hp::SpecModule *sm = nullptr;
    const int rc = hp::spec_get(S->ctx->device, R->spec_src, &sm, log);
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return;  // the worker has failed every queued request
    S->to_compile.pop_front();
    if (rc) {
      R->done = R->failed = true;
      R->error = "specialised kernel: " + std::string(hipGetErrorString((hipError_t)rc)) +
                 (log.empty() ? "" : "\n" + log);
      S->cv_done.notify_all();
    } else {
      R->sm = sm;
      R->spec_src.clear();
      R->spec_src.shrink_to_fit();
      S->pending.push_back(R);
      S->cv_work.notify_one();
    }
  }
}

}  // namespace

extern "C" {

int hp_server_create(hp_context *ctx, size_t hbm_budget_bytes, hp_server **out) {
  if (!ctx || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (hbm_budget_bytes < slot_bytes() * kMinChunk)
    return fail(HP_E_BUDGET, "budget below one chunk of " + std::to_string(kMinChunk) + " paths");
  HIP_TRY(hipSetDevice(ctx->device));
  std::unique_ptr<hp_server> S(new hp_server());
  S->ctx = ctx;
  S->budget = hbm_budget_bytes;
  // arena sized by the budget (in path slots of the widest system)
  S->arena_paths = (int64_t)(hbm_budget_bytes / slot_bytes());
  int rc;
  if ((rc = S->a_ends.alloc((size_t)S->arena_paths * HP_MAX_N * sizeof(hp_c64)))) return rc;
  if ((rc = S->a_status.alloc((size_t)S->arena_paths * sizeof(int32_t)))) return rc;
  if ((rc = S->a_stats.alloc((size_t)S->arena_paths * sizeof(hp_path_stats)))) return rc;
  S->free_list.push_back({0, S->arena_paths});
  HIP_TRY(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
  for (int f = 0; f < kFamilyStreams; ++f)
    HIP_TRY(hipStreamCreateWithFlags(&S->fam_stream[f], hipStreamNonBlocking));
  // no slot holds a path yet
  HIP_TRY((hipError_t)hp_launch_fill_i32(S->a_status.as<int32_t>(), S->arena_paths, hp::kUnstarted,
                                         S->stream));
  HIP_TRY(hipStreamSynchronize(S->stream));
  hp_server *raw = S.get();
  S->worker = std::thread(worker_main, raw);
  S->compiler = std::thread(compiler_main, raw);
  context_adopt(ctx);
  *out = S.release();
  return HP_OK;
}

int hp_server_set_slice(hp_server *S, double slice_ms, int32_t fixed_steps) {
  if (!S) return fail(HP_E_INVALID_ARG, "NULL server");
  if (!(slice_ms >= 0.0) || !std::isfinite(slice_ms) || fixed_steps < 0)
    return fail(HP_E_INVALID_ARG, "slice_ms must be finite and >= 0, fixed_steps >= 0");
  std::lock_guard<std::mutex> lk(S->mu);
  S->slice_ms = slice_ms;
  S->fixed_steps = fixed_steps;
  S->fam_budget.clear();
  return HP_OK;
}

int hp_server_info_get(hp_server *S, hp_server_info *out) {
  if (!S || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  std::memset(out, 0, sizeof(*out));
  out->epochs = S->epochs;
  out->carried = S->carried;
  out->epoch_ms_max = S->epoch_ms_max;
  out->epoch_ms_mean = S->epochs ? S->epoch_ms_sum / (double)S->epochs : 0.0;
  out->slice_ms = S->slice_ms;
  out->fixed_steps = S->fixed_steps;
  int32_t bmin = 0, bmax = 0;
  for (auto &b : S->fam_budget) {
    bmin = bmin ? std::min(bmin, b.second) : b.second;
    bmax = std::max(bmax, b.second);
  }
  out->budget_min = bmin;
  out->budget_max = bmax;
  out->peak_bytes = S->peak;
  return HP_OK;
}

int hp_server_submit(hp_server *S, const hp_system *f, hp_c64 gamma, const hp_tolerances *tol,
                     int64_t *req_id) {
  if (!S || !req_id) return fail(HP_E_INVALID_ARG, "NULL argument");
  auto R = std::make_shared<Request>();
  int rc = check_system(f, R->info);
  if (rc) return rc;
  if ((rc = check_tol(tol))) return rc;
  if (!std::isfinite(gamma.re) || !std::isfinite(gamma.im) || (gamma.re == 0 && gamma.im == 0))
    return fail(HP_E_INVALID_ARG, "gamma must be finite and nonzero");
  const int n = f->n;
  {
    // the request must fit the variant chosen for it alone; a mixed launch
    // takes the widest variant of its requests, which fits as well
    Packed one;
    pack_append(one, f, R->info, gamma, 1, 0, 0, nullptr);
    const Kv kv = kv_pick(one);
    if (kv.nmax < n) return fail(HP_E_UNSUPPORTED_N, "no kernel variant for n");
    if ((rc = check_lds(S->ctx, kv_lds(kv, one)))) return rc;
    R->dense_code = kv.dense ? kv.code : 0;
    // systems a specialised kernel serves run on it (compiled on the
    // server's compile thread the first time their support is seen, then
    // shared by every request of that support)
    const DevSys &d = one.sys[0];
    if (!R->dense_code && hp::spec_eligible(n, one.terms.data(), d.n_terms))
      R->spec_src = hp::spec_source(n, d.deg, one.terms.data(), d.n_terms, true);
  }
  R->eq_ptr.assign(f->eq_ptr, f->eq_ptr + n + 1);
  R->coeff.assign(f->coeff, f->coeff + f->n_terms);
  R->exps.assign(f->exps, f->exps + (size_t)f->n_terms * n);
  R->sys = hp_system{n, f->n_terms, R->eq_ptr.data(), R->coeff.data(), R->exps.data()};
  R->gamma = gamma;
  if (tol) R->tol = *tol;
  else hp_default_tolerances(&R->tol);
  R->ends.resize((size_t)R->info.paths * n);
  R->status.resize(R->info.paths);
  R->stats.resize(R->info.paths);
  R->t_submit = now_ms();
  std::lock_guard<std::mutex> lk(S->mu);
  R->id = S->next_id++;
  S->all[R->id] = R;
  if (R->spec_src.empty()) {
    S->pending.push_back(R);
    S->cv_work.notify_one();
  } else {
    S->to_compile.push_back(R);
    S->cv_compile.notify_one();
  }
  *req_id = R->id;
  return HP_OK;
}

int hp_server_poll(hp_server *S, int64_t req_id, int32_t *done) {
  if (!S || !done) return fail(HP_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return fail(HP_E_INVALID_ARG, "unknown request id");
  *done = it->second->done ? 1 : 0;
  return HP_OK;
}

int hp_server_wait(hp_server *S, int64_t req_id, hp_c64 *endpoints, int32_t *status,
                   hp_path_stats *stats, double *latency_ms) {
  if (!S) return fail(HP_E_INVALID_ARG, "NULL server");
  std::shared_ptr<Request> R;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(req_id);
    if (it == S->all.end()) return fail(HP_E_INVALID_ARG, "unknown request id");
    R = it->second;
    S->cv_done.wait(lk, [&] { return R->done; });
    S->all.erase(it);
    if (R->failed) return fail(HP_E_DEVICE, "request failed: " + (R->error.empty() ? S->error : R->error));
  }
  if (endpoints) std::memcpy(endpoints, R->ends.data(), R->ends.size() * sizeof(hp_c64));
  if (status) std::memcpy(status, R->status.data(), R->status.size() * sizeof(int32_t));
  if (stats) std::memcpy(stats, R->stats.data(), R->stats.size() * sizeof(hp_path_stats));
  if (latency_ms) *latency_ms = R->t_done - R->t_submit;
  return HP_OK;
}

int hp_server_peak_bytes(hp_server *S, size_t *out) {
  if (!S || !out) return fail(HP_E_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->peak;
  return HP_OK;
}

void hp_server_destroy(hp_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
    S->cv_compile.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  if (S->compiler.joinable()) S->compiler.join();
  (void)hipSetDevice(S->ctx->device);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (int f = 0; f < kFamilyStreams; ++f)
    if (S->fam_stream[f]) (void)hipStreamSynchronize(S->fam_stream[f]);
  for (auto &ev : S->fam_ev)
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  for (int f = 0; f < kFamilyStreams; ++f)
    if (S->fam_stream[f]) (void)hipStreamDestroy(S->fam_stream[f]);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  hp_context *ctx = S->ctx;
  delete S;
  context_orphan(ctx);
}

}  // extern "C"

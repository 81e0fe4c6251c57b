// Kernels specialised at run time to one polynomial system: the evaluator
// of H and its Jacobian is written out as straight-line HIP for the
// system's support (term structure, exponents, start-system degrees), put
// together with the one-path-per-lane tracker (spec_track.hpp) and compiled
// for gfx950 through hiprtc.  Coefficients, gamma, tolerances and start
// points stay run-time data, so one compiled module serves every system with
// the same support.
#include "hp_jit.hpp"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <utility>

namespace hp {

namespace {

// Text of the headers the generated source includes (written by the build
// from the library's own headers).
#include "hp_jit_headers.inc"

// hiprtc has no C library headers; these stand in for the two the shared
// headers include (hiprtc itself defines size_t).
const char kRtcStdint[] =
    "#pragma once\n"
    "typedef signed char int8_t;\ntypedef unsigned char uint8_t;\n"
    "typedef short int16_t;\ntypedef unsigned short uint16_t;\n"
    "typedef int int32_t;\ntypedef unsigned int uint32_t;\n"
    "typedef long int64_t;\ntypedef unsigned long uint64_t;\n";
const char kRtcStddef[] = "#pragma once\n";

struct Factor {
  int v, e;
};
struct GenTerm {
  int eq;
  std::vector<Factor> f;
};

GenTerm unpack(const DevTerm &T) {
  uint8_t bytes[16];
  std::memcpy(bytes, T.w, 16);
  GenTerm g;
  g.eq = bytes[15];
  const int k = bytes[0] & 0x7f;
  for (int m = 0; m < k; ++m) g.f.push_back({bytes[1 + m] & 15, bytes[1 + m] >> 4});
  return g;
}

std::string pw(int v, int e) { return "p" + std::to_string(v) + "_" + std::to_string(e); }
std::string jn(int i, int j) { return "J[" + std::to_string(i) + "][" + std::to_string(j) + "]"; }

}  // namespace

bool spec_eligible(int n, const DevTerm *terms, int n_terms) {
  if (n < 1 || n > kSpecMaxN) return false;
  int64_t factors = 0;
  for (int t = 0; t < n_terms; ++t) factors += (int64_t)unpack(terms[t]).f.size();
  return factors <= kSpecMaxFactors;
}

// Coefficient-parameter form (the start system g has f's support, term by
// term): with s = gamma (1 - t), H = sum_k (s cg_k + t cf_k) x^a_k, so one
// sweep over the monomials with the blended coefficient b_k = s cg_k + t cf_k
// gives J = sum_k b_k grad x^a_k and the value H; the right-hand side
// -H_t = sum_k (gamma cg_k - cf_k) x^a_k takes the third coefficient of the
// term instead (and at t = 1, b_k = cf_k gives f).  Per term, prefix
// products of the bare monomial give its value; a backward sweep of suffix
// products that starts from b_k gives the partial derivatives.  The
// coefficient table holds (cf_k, cg_k, gamma cg_k - cf_k) per term.
std::string param_source(int n, const DevTerm *terms, int n_terms) {
  std::vector<GenTerm> T;
  T.reserve(n_terms);
  std::vector<int> emax(n, 1);
  for (int t = 0; t < n_terms; ++t) {
    T.push_back(unpack(terms[t]));
    for (const Factor &f : T.back().f) emax[f.v] = std::max(emax[f.v], f.e);
  }
  std::ostringstream o;
  o << "#include \"spec_track.hpp\"\n\nnamespace hp {\nnamespace gen {\n\nstruct Sys {\n"
    << "  static constexpr int N = " << n << ";\n"
    << "  static constexpr bool kParam = true;\n"
    << "  __device__ __forceinline__ static void eval(cptr<double2> cf, const cd (&x)[N], double te,\n"
    << "                                              cd s, cd gamma, int emode, cd (&J)[N][N],\n"
    << "                                              lds_char *spare) {\n"
    << "    const bool rhs_t = (emode == EV_NEG_HT);\n";
  for (int v = 0; v < n; ++v) {
    o << "    const cd " << pw(v, 1) << " = x[" << v << "];\n";
    for (int e = 2; e <= emax[v]; ++e)
      o << "    const cd " << pw(v, e) << " = cmul(" << pw(v, e - 1) << ", x[" << v << "]);\n";
  }
  o << "    cd F[N];\n";
  std::vector<char> jt((size_t)n * n, 0), ft(n, 0);
  std::vector<int> last(n, -1);
  for (int t = 0; t < n_terms; ++t) last[T[t].eq] = t;
  auto slot = [](int i) { return "spare + " + std::to_string(i * 1024); };
  auto add_f = [&](int eq, const std::string &val) {
    const std::string fe = "F[" + std::to_string(eq) + "]";
    if (ft[eq]) o << "      " << fe << " = cadd(" << fe << ", " << val << ");\n";
    else o << "      " << fe << " = " << val << ";\n";
    ft[eq] = 1;
  };
  for (int t = 0; t < n_terms; ++t) {
    const GenTerm &g = T[t];
    const int K = (int)g.f.size();
    o << "    {\n      const double2 f_ = cf[" << 3 * t << "], g_ = cf[" << 3 * t + 1 << "], d_ = cf["
      << 3 * t + 2 << "];\n"
      << "      const cd b = cadd(cmul(s, cd{g_.x, g_.y}), cscale(cd{f_.x, f_.y}, te));\n"
      << "      const cd r = csel(rhs_t, cd{d_.x, d_.y}, b);\n";
    if (K == 0) {
      add_f(g.eq, "r");
      o << "    }\n";
      if (last[g.eq] == t) o << "    stl(" << slot(g.eq) << ", F[" << g.eq << "]);\n";
      continue;
    }
    // prefix products of the bare monomial: m0 = x^e0, m_j = m_{j-1} x^ej
    for (int m = 1; m < K; ++m)
      o << "      const cd m" << m << " = cmul(" << (m == 1 ? pw(g.f[0].v, g.f[0].e) : "m" + std::to_string(m - 1))
        << ", " << pw(g.f[m].v, g.f[m].e) << ");\n";
    const std::string mono = K == 1 ? pw(g.f[0].v, g.f[0].e) : "m" + std::to_string(K - 1);
    add_f(g.eq, "cmul(r, " + mono + ")");
    // backward sweep: S = b times the product of the factors after m
    for (int m = K - 1; m >= 0; --m) {
      const int v = g.f[m].v, e = g.f[m].e;
      const std::string left = (m == 0) ? "" : (m == 1 ? pw(g.f[0].v, g.f[0].e) : "m" + std::to_string(m - 1));
      const std::string suf = (m == K - 1) ? "b" : "S";
      const std::string je = jn(g.eq, v);
      const bool first = !jt[(size_t)g.eq * n + v];
      jt[(size_t)g.eq * n + v] = 1;
      std::string d = left.empty() ? suf : "cmul(" + left + ", " + suf + ")";
      if (e > 1) d = "cmul(" + d + ", cscale(" + pw(v, e - 1) + ", " + std::to_string(e) + ".0))";
      if (first) o << "      " << je << " = " << d << ";\n";
      else if (e == 1 && !left.empty()) o << "      " << je << " = cfma(" << je << ", " << left << ", " << suf << ");\n";
      else o << "      " << je << " = cadd(" << je << ", " << d << ");\n";
      if (m > 0) {
        if (m == K - 1) o << "      cd S = cmul(" << pw(v, e) << ", b);\n";
        else o << "      S = cmul(S, " << pw(v, e) << ");\n";
      }
    }
    o << "    }\n";
    if (last[g.eq] == t) o << "    stl(" << slot(g.eq) << ", F[" << g.eq << "]);\n";
  }
  for (int i = 0; i < n; ++i) {
    if (!ft[i]) o << "    stl(" << slot(i) << ", cd{0.0, 0.0});\n";
    for (int j = 0; j < n; ++j)
      if (!jt[(size_t)i * n + j]) o << "    " << jn(i, j) << " = {0.0, 0.0};\n";
  }
  o << "  }\n};\n\n}  // namespace gen\n}  // namespace hp\n\n"
    << "using SpecT = hp::Spec<hp::gen::Sys>;\n"
    << "constexpr int kRkBytes = hp::RkLds<hp::gen::Sys::N>::kBytes;\n\n"
    << "extern \"C\" __global__ void __launch_bounds__(64) hp_spec_persistent(hp::KArgs a) {\n"
    << "  __shared__ __attribute__((aligned(16))) char rk[kRkBytes];\n"
    << "  SpecT tr(a, (hp::lds_char *)rk);\n  hp::lane_persistent<false>(a, tr);\n}\n\n"
    << "extern \"C\" __global__ void __launch_bounds__(64) hp_spec_plain(hp::KArgs a) {\n"
    << "  __shared__ __attribute__((aligned(16))) char rk[kRkBytes];\n"
    << "  SpecT tr(a, (hp::lds_char *)rk);\n  hp::lane_plain<SpecT, 64>(a, tr);\n}\n";
  return o.str();
}

// The evaluator follows the group and lane kernels term by term: prefix
// products from the coefficient give the term value; a backward sweep of
// suffix products that starts from t gives its partial derivatives already
// scaled by t (times e x_v^{e-1} for an exponent e > 1).  The start system
// adds s d_i x_i^{d_i-1} on the diagonal; the right-hand side is chosen by
// emode.  A Jacobian entry or value is assigned at its first contribution
// and accumulated with fused multiply-adds afterwards.
std::string spec_source(int n, const int32_t *deg, const DevTerm *terms, int n_terms, bool sliced,
                        bool param) {
  if (param) return param_source(n, terms, n_terms);
  std::vector<GenTerm> T;
  T.reserve(n_terms);
  std::vector<int> emax(n, 1);  // powers the terms use (computed up front)
  for (int t = 0; t < n_terms; ++t) {
    T.push_back(unpack(terms[t]));
    for (const Factor &f : T.back().f) emax[f.v] = std::max(emax[f.v], f.e);
  }
  std::ostringstream o;
  o << "#include \"spec_track.hpp\"\n\nnamespace hp {\nnamespace gen {\n\nstruct Sys {\n"
    << "  static constexpr int N = " << n << ";\n"
    << "  static constexpr bool kParam = false;\n"
    << "  __device__ __forceinline__ static void eval(cptr<double2> cf, const cd (&x)[N], double te,\n"
    << "                                              cd s, cd gamma, int emode, cd (&J)[N][N],\n"
    << "                                              lds_char *spare) {\n";
  for (int v = 0; v < n; ++v) {
    o << "    const cd " << pw(v, 1) << " = x[" << v << "];\n";
    for (int e = 2; e <= emax[v]; ++e)
      o << "    const cd " << pw(v, e) << " = cmul(" << pw(v, e - 1) << ", x[" << v << "]);\n";
  }
  o << "    cd F[N];\n";
  std::vector<char> jt((size_t)n * n, 0), ft(n, 0);
  // an equation's value goes to the lane's spare LDS slot after its last
  // term (out of the registers the Jacobian needs), its right-hand side
  // replaces it there at the end
  std::vector<int> last(n, -1);
  for (int t = 0; t < n_terms; ++t) last[T[t].eq] = t;
  auto slot = [](int i) { return "spare + " + std::to_string(i * 1024); };
  auto add_f = [&](int eq, const std::string &val) {
    const std::string fe = "F[" + std::to_string(eq) + "]";
    if (ft[eq]) o << "      " << fe << " = cadd(" << fe << ", " << val << ");\n";
    else o << "      " << fe << " = " << val << ";\n";
    ft[eq] = 1;
  };
  for (int t = 0; t < n_terms; ++t) {
    const GenTerm &g = T[t];
    const int K = (int)g.f.size();
    o << "    {\n      const double2 c_ = cf[" << t << "];\n      const cd c = {c_.x, c_.y};\n";
    if (K == 0) {
      add_f(g.eq, "c");
      o << "    }\n";
      if (last[g.eq] == t) o << "    stl(" << slot(g.eq) << ", F[" << g.eq << "]);\n";
      continue;
    }
    for (int m = 0; m < K; ++m)
      o << "      const cd q" << m << " = cmul(" << (m == 0 ? std::string("c") : "q" + std::to_string(m - 1))
        << ", " << pw(g.f[m].v, g.f[m].e) << ");\n";
    add_f(g.eq, "q" + std::to_string(K - 1));
    for (int m = K - 1; m >= 0; --m) {
      const int v = g.f[m].v, e = g.f[m].e;
      const std::string left = (m == 0) ? "c" : "q" + std::to_string(m - 1);
      const std::string je = jn(g.eq, v);
      const bool first = !jt[(size_t)g.eq * n + v];
      jt[(size_t)g.eq * n + v] = 1;
      if (e > 1) {
        const std::string d = (m == K - 1) ? "cscale(" + left + ", te)" : "cmul(" + left + ", S)";
        const std::string de = "cmul(" + d + ", cscale(" + pw(v, e - 1) + ", " + std::to_string(e) + ".0))";
        if (first) o << "      " << je << " = " << de << ";\n";
        else o << "      " << je << " = cadd(" << je << ", " << de << ");\n";
      } else if (m == K - 1) {
        if (first) o << "      " << je << " = cscale(" << left << ", te);\n";
        else o << "      " << je << " = cfma_r(" << je << ", " << left << ", te);\n";
      } else {
        if (first) o << "      " << je << " = cmul(" << left << ", S);\n";
        else o << "      " << je << " = cfma(" << je << ", " << left << ", S);\n";
      }
      if (m > 0) {
        if (m == K - 1) o << "      cd S = cscale(" << pw(v, e) << ", te);\n";
        else o << "      S = cmul(S, " << pw(v, e) << ");\n";
      }
    }
    o << "    }\n";
    if (last[g.eq] == t) o << "    stl(" << slot(g.eq) << ", F[" << g.eq << "]);\n";
  }
  for (int i = 0; i < n; ++i) {
    if (!ft[i]) o << "    stl(" << slot(i) << ", cd{0.0, 0.0});\n";
    for (int j = 0; j < n; ++j)
      if (!jt[(size_t)i * n + j]) o << "    " << jn(i, j) << " = {0.0, 0.0};\n";
  }
  o << "    asm volatile(\"\" ::: \"memory\");  // values are reloaded, not kept in registers\n";
  // start system x_i^{d_i} - 1 and the right-hand side; the powers x_i^e,
  // e < d_i, are formed here (live only in this block) by the same chain of
  // products as the term powers
  for (int i = 0; i < n; ++i) {
    const int d = deg[i];
    const std::string xi = "x[" + std::to_string(i) + "]";
    o << "    {\n";
    if (d == 1) {
      o << "      const cd xq = cd{1.0, 0.0};\n";
    } else {
      o << "      cd xq = " << xi << ";\n";
      for (int e = 2; e < d; ++e) o << "      xq = cmul(xq, " << xi << ");\n";
    }
    o << "      cd g = cmul(xq, " << xi << ");\n"
      << "      g.re -= 1.0;\n"
      << "      " << jn(i, i) << " = cadd(" << jn(i, i) << ", cmul(s, cscale(xq, " << d << ".0)));\n"
      << "      const cd f = ldl(" << slot(i) << ");\n"
      << "      const cd hv = cadd(cmul(s, g), cscale(f, te));\n"
      << "      const cd mht = csub(cmul(gamma, g), f);\n"
      << "      stl(" << slot(i) << ", csel(emode == EV_F, f, csel(emode == EV_H, hv, mht)));\n"
      << "    }\n";
  }
  o << "  }\n};\n\n}  // namespace gen\n}  // namespace hp\n\n"
    << "using SpecT = hp::Spec<hp::gen::Sys>;\n"
    << "constexpr int kRkBytes = hp::RkLds<hp::gen::Sys::N>::kBytes;\n\n"
    << "extern \"C\" __global__ void __launch_bounds__(64) hp_spec_persistent(hp::KArgs a) {\n"
    << "  __shared__ __attribute__((aligned(16))) char rk[kRkBytes];\n"
    << "  SpecT tr(a, (hp::lds_char *)rk);\n  hp::lane_persistent<" << (sliced ? "true" : "false")
    << ">(a, tr);\n}\n";
  // the serving form (sliced) has no plain kernel
  if (!sliced)
    o << "\nextern \"C\" __global__ void __launch_bounds__(64) hp_spec_plain(hp::KArgs a) {\n"
      << "  __shared__ __attribute__((aligned(16))) char rk[kRkBytes];\n"
      << "  SpecT tr(a, (hp::lds_char *)rk);\n  hp::lane_plain<SpecT, 64>(a, tr);\n}\n";
  return o.str();
}

namespace {

// Code objects already built in this process, by source.
std::mutex g_code_mu;
std::map<std::string, std::vector<char>> g_code;

// hiprtc options of every specialised kernel (no packed FP32 instructions in
// device code, as for the compiled kernels).
const char *const kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                                "-target-feature", "-Xclang", "-packed-fp32-ops"};

// What a cached code object depends on besides its source: the compiler
// version and options, and the text of the headers the source includes (a
// 64-bit FNV-1a digest of their names and texts).
std::string build_tag() {
  static const std::string tag = [] {
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    std::string t = "hiprtc " + std::to_string(major) + "." + std::to_string(minor);
    for (const char *o : kRtcOpts) t += std::string(" ") + o;
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&h](const char *s) {
      // each string ends with a 0xff byte, which no header text holds
      for (;; ++s) {
        h ^= *s ? (unsigned char)*s : 0xffu;
        h *= 0x100000001b3ull;
        if (!*s) break;
      }
    };
    for (size_t i = 0; i < sizeof(kJitHeaderNames) / sizeof(kJitHeaderNames[0]); ++i) {
      mix(kJitHeaderNames[i]);
      mix(kJitHeaderTexts[i]);
    }
    mix(kRtcStdint);
    mix(kRtcStddef);
    char d[40];
    std::snprintf(d, sizeof(d), " headers %016llx", (unsigned long long)h);
    return t + d + "\n";
  }();
  return tag;
}

// File of the on-disk code cache ($HP_JIT_CACHE, when set): named by a hash
// of the key (build tag + source); the file starts with the key itself, so
// that a hash collision or another compiler reads as a miss.
std::string disk_path(const std::string &key) {
  const char *dir = std::getenv("HP_JIT_CACHE");
  if (!dir || !*dir) return std::string();
  char name[40];
  std::snprintf(name, sizeof(name), "/hp_spec_%016zx.bin", std::hash<std::string>()(key));
  return std::string(dir) + name;
}

bool disk_load(const std::string &src, std::vector<char> &code) {
  const std::string key = build_tag() + src;
  const std::string path = disk_path(key);
  if (path.empty()) return false;
  std::ifstream in(path, std::ios::binary);
  if (!in) return false;
  uint64_t ls = 0, lc = 0;
  in.read((char *)&ls, sizeof(ls));
  if (!in || ls != key.size()) return false;
  std::string s2(ls, '\0');
  in.read(&s2[0], (std::streamsize)ls);
  in.read((char *)&lc, sizeof(lc));
  if (!in || s2 != key || lc == 0 || lc > (1ull << 30)) return false;
  code.resize(lc);
  in.read(code.data(), (std::streamsize)lc);
  return (bool)in;
}

void disk_store(const std::string &src, const std::vector<char> &code) {
  static std::atomic<unsigned> seq{0};
  const std::string key = build_tag() + src;
  const std::string path = disk_path(key);
  if (path.empty()) return;
  const std::string tmp =
      path + ".tmp" + std::to_string((long)getpid()) + "_" + std::to_string(seq++);
  {
    std::ofstream out(tmp, std::ios::binary);
    if (!out) return;
    const uint64_t ls = key.size(), lc = code.size();
    out.write((const char *)&ls, sizeof(ls));
    out.write(key.data(), (std::streamsize)ls);
    out.write((const char *)&lc, sizeof(lc));
    out.write(code.data(), (std::streamsize)lc);
    if (!out) {
      std::remove(tmp.c_str());
      return;
    }
  }
  std::rename(tmp.c_str(), path.c_str());  // readers see a whole file or none
}

int rtc_compile(const std::string &src, std::vector<char> &code, std::string &log) {
  std::vector<const char *> names, texts;
  for (size_t i = 0; i < sizeof(kJitHeaderNames) / sizeof(kJitHeaderNames[0]); ++i) {
    names.push_back(kJitHeaderNames[i]);
    texts.push_back(kJitHeaderTexts[i]);
  }
  names.push_back("stdint.h");
  texts.push_back(kRtcStdint);
  names.push_back("stddef.h");
  texts.push_back(kRtcStddef);
  hiprtcProgram prog;
  hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "hp_spec.hip", (int)names.size(),
                                       texts.data(), names.data());
  if (r != HIPRTC_SUCCESS) {
    log = hiprtcGetErrorString(r);
    return (int)hipErrorInvalidValue;
  }
  r = hiprtcCompileProgram(prog, (int)(sizeof(kRtcOpts) / sizeof(kRtcOpts[0])), kRtcOpts);
  size_t ls = 0;
  hiprtcGetProgramLogSize(prog, &ls);
  log.assign(ls, '\0');
  if (ls) hiprtcGetProgramLog(prog, &log[0]);
  int rc = (int)hipSuccess;
  if (r != HIPRTC_SUCCESS) {
    rc = (int)hipErrorInvalidImage;
  } else {
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code.resize(cs);
    if (cs == 0 || hiprtcGetCode(prog, code.data()) != HIPRTC_SUCCESS) rc = (int)hipErrorInvalidImage;
  }
  hiprtcDestroyProgram(&prog);
  return rc;
}

}  // namespace

int spec_compile(const std::string &src, std::vector<char> &code, std::string &log) {
  {
    std::lock_guard<std::mutex> g(g_code_mu);
    auto it = g_code.find(src);
    if (it != g_code.end()) {
      code = it->second;
      return (int)hipSuccess;
    }
  }
  if (!disk_load(src, code)) {
    const int rc = rtc_compile(src, code, log);
    if (rc) return rc;
    disk_store(src, code);
  }
  std::lock_guard<std::mutex> g(g_code_mu);
  g_code.emplace(src, code);
  return (int)hipSuccess;
}

int spec_get(int device, const std::string &src, const SpecModule **out, std::string &log) {
  static std::mutex mu;
  static std::map<std::pair<int, std::string>, std::unique_ptr<SpecModule>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(device, src);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *out = it->second.get();
    return (int)hipSuccess;
  }
  std::vector<char> code;
  int rc = spec_compile(src, code, log);
  if (rc) return rc;
  std::unique_ptr<SpecModule> m(new SpecModule());
  hipError_t e = hipModuleLoadData(&m->mod, code.data());
  if (e == hipSuccess) e = hipModuleGetFunction(&m->persistent, m->mod, "hp_spec_persistent");
  // a serving (sliced) module has no plain kernel
  if (e == hipSuccess && src.find("hp_spec_plain") != std::string::npos)
    e = hipModuleGetFunction(&m->plain, m->mod, "hp_spec_plain");
  if (e != hipSuccess) {
    if (m->mod) (void)hipModuleUnload(m->mod);
    return (int)e;
  }
  *out = m.get();
  cache.emplace(std::move(key), std::move(m));
  return (int)hipSuccess;
}

}  // namespace hp

// Kernels specialised at run time to one polynomial system (host side):
// source generation, hiprtc compilation and a per-process module cache.
// Not part of the C ABI.
#pragma once

#include <string>
#include <vector>

#include "hp_internal.hpp"

namespace hp {

// Largest n of a specialised kernel: its [J | rhs] lives in registers
// (n = 9, 10 spill part of it to scratch and still run several times faster
// than the group kernels; from n = 11 on the spills make them slower).
constexpr int kSpecMaxN = 10;
// Largest total factor count (sum over terms of the factors) of a system
// with a specialised kernel; bounds its code size and compile time.
constexpr int kSpecMaxFactors = 1024;

// True when a system of n unknowns with these packed terms (the total-degree
// start system) can have a specialised kernel.
bool spec_eligible(int n, const DevTerm *terms, int n_terms);

// HIP source of the specialised kernels hp_spec_persistent and hp_spec_plain
// for a system of n unknowns, start-system degrees deg[0..n-1] and terms in
// packed order (sorted by factor count; the coefficients stay run-time data).
// sliced: the serving form, whose persistent kernel suspends and resumes
// paths (lane_drain) and which has no plain kernel
// param: the coefficient-parameter form (a start system on f's support,
// coefficient table of (f, g, gamma g - f) per term, start points from
// memory; plans only)
std::string spec_source(int n, const int32_t *deg, const DevTerm *terms, int n_terms,
                        bool sliced = false, bool param = false);

// Code object of spec source for gfx950 (no device needed): from this
// process's cache, else from the directory $HP_JIT_CACHE names (when set),
// else compiled through hiprtc and stored in both.  The compiler log goes to
// `log`.  hipSuccess or an error.
int spec_compile(const std::string &src, std::vector<char> &code, std::string &log);

// Loaded specialised kernels of one system on one device.
struct SpecModule {
  hipModule_t mod = nullptr;
  hipFunction_t persistent = nullptr;
  hipFunction_t plain = nullptr;
};

// Module for `src` on the current device, compiled and loaded at its first
// request and kept until the process ends.  hipSuccess or an error (log in
// `log`).
int spec_get(int device, const std::string &src, const SpecModule **out, std::string &log);

}  // namespace hp

// burn_codegen.h -- host side of the per-network code generation: the
// generated source, its compilation for gfx950 with hiprtc, and the cache
// of compiled code objects.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace bn {

// A network as the generator sees it (host copies of bn_network_desc).
struct GenDesc {
  int N = 0, R = 0;
  std::vector<int> mass, reac, prod;  // [N], [3R], [3R]
  std::vector<double> coef, q;        // [7R], [R]
  double c_v = 1.0;
};

// Lanes per cell the generated body supports for a system of n components:
// one lane up to GEN_MAX_N1, two up to GEN_MAX_N2 (the LU rows of a lane
// stay in its registers).
constexpr int GEN_MAX_N1 = 8;
constexpr int GEN_MAX_N2 = 16;

// Row patterns (bit j: column j) of the Jacobian and of the LU factors of
// I - cJ with diagonal pivots.
void jac_pattern(const GenDesc &d, std::vector<unsigned long long> *pat);
void fill_pattern(const GenDesc &d, std::vector<unsigned long long> *fill);

// The generated source (network part; it includes burn_gen_body.h).
std::string gen_source(const GenDesc &d, int lpc);
// Jacobian entries stored per lane (the workspace's rows).
int gen_entries(const GenDesc &d, int lpc);
// Dynamic LDS of a workgroup of four waves.
size_t gen_lds_bytes(const GenDesc &d, int lpc);
// Cache key of a source (with the body, the options and the compiler version).
uint64_t gen_key(const std::string &src);
// Source -> code object; cache_dir may be empty (no cache).  0 or -1 (err set).
int gen_build(const GenDesc &d, int lpc, const std::string &cache_dir, std::vector<char> *code,
              std::string *err);

}  // namespace bn

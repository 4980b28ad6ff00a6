// burn_codegen.cpp -- per-network code generation (Sec. 2 of the paper: the
// network's right-hand side and analytic Jacobian are generated for each
// network) and its run-time compilation for gfx950.
//
// The generated source defines struct bng::GenNet (sizes, the LU fill
// pattern of I - cJ with diagonal pivots, and the straight-line rates,
// right-hand side and Jacobian of the network) and the kernel bn_gen_burn;
// the integrator itself is burn_gen_body.h, compiled with it.  Each
// quantity is evaluated with the operations of its definition in a fixed
// order (rates as lambda(T) e^{p} / prod m! rho^{n-1} prod Y, species sums in
// ascending reaction order, the heat term divided by c_v, Jacobian terms
// slot by slot in ascending reaction order) and without contraction, so a
// serial FP64 evaluation of the same definitions rounds the same way up to
// the exp / log / cbrt implementations and one choice: the exponent of a
// rate, a0 + a1/T + ... + a6 ln T, is summed in the same order with fused
// multiply-adds (six instead of twelve operations per rate; its rounding
// differs from the serial sum by a few units in the last place, as the
// exponential's implementations do).

#include "burn_codegen.h"

#include <hip/hiprtc.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <iterator>
#include <sys/stat.h>
#include <unistd.h>

namespace bn {
namespace {

#include "burn_gen_headers.inc"  // BNG_BODY_H, BNG_ARGS_H, BNG_MATH_H: the headers' text

std::string hexd(double v) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "%a", v);
  return std::string("(") + buf + ")";
}

int nu_of(const GenDesc &d, int i, int r) {
  int v = 0;
  for (int s = 0; s < 3; ++s) {
    v += (d.prod[3 * r + s] == i);
    v -= (d.reac[3 * r + s] == i);
  }
  return v;
}

// 1 / prod over distinct reactant species of (multiplicity)!, and the
// number of reactant slots in use
double inv_fact(const GenDesc &d, int r, int *nr) {
  const int *s = d.reac.data() + 3 * r;
  double f = 1.0;
  int cnt = 0;
  for (int i = 0; i < 3; ++i) {
    if (s[i] < 0) continue;
    ++cnt;
    bool first = true;
    for (int j = 0; j < i; ++j)
      if (s[j] == s[i]) first = false;
    if (!first) continue;
    int m = 0;
    for (int j = 0; j < 3; ++j) m += (s[j] == s[i]);
    for (int j = 2; j <= m; ++j) f *= (double)j;
  }
  *nr = cnt;
  return 1.0 / f;
}

// term "w * x" of a sum with integer weight w (w * x is exact for |w| <= 2)
std::string wterm(int w, const std::string &x) {
  if (w == 1) return x;
  if (w == -1) return "(-" + x + ")";
  return "(" + std::to_string(w) + ".0 * " + x + ")";
}

}  // namespace

void jac_pattern(const GenDesc &d, std::vector<unsigned long long> *pat) {
  const int N = d.N, n = N + 1;
  pat->assign(n, 0ull);
  for (int r = 0; r < d.R; ++r) {
    for (int i = 0; i < N; ++i) {
      if (!nu_of(d, i, r)) continue;
      for (int a = 0; a < 3; ++a)
        if (d.reac[3 * r + a] >= 0) (*pat)[i] |= 1ull << d.reac[3 * r + a];
      (*pat)[i] |= 1ull << N;
    }
    for (int a = 0; a < 3; ++a)
      if (d.reac[3 * r + a] >= 0) (*pat)[N] |= 1ull << d.reac[3 * r + a];
    (*pat)[N] |= 1ull << N;
  }
}

void fill_pattern(const GenDesc &d, std::vector<unsigned long long> *fill) {
  const int n = d.N + 1;
  jac_pattern(d, fill);
  for (int i = 0; i < n; ++i) (*fill)[i] |= 1ull << i;
  for (int K = 0; K < n; ++K) {
    const unsigned long long above = ~((2ull << K) - 1ull);  // columns > K
    for (int i = K + 1; i < n; ++i)
      if (((*fill)[i] >> K) & 1ull) (*fill)[i] |= (*fill)[K] & above;
  }
}

std::string gen_source(const GenDesc &d, int lpc) {
  const int N = d.N, R = d.R, n = N + 1;
  const int NS = (n + lpc - 1) / lpc;
  std::vector<unsigned long long> jp, fp;
  jac_pattern(d, &jp);
  fill_pattern(d, &fp);
  std::vector<unsigned long long> ujp(NS, 0), ufp(NS, 0);
  for (int s = 0; s < NS; ++s)
    for (int hh = 0; hh < lpc; ++hh) {
      const int i = s * lpc + hh;
      if (i < n) {
        ujp[s] |= jp[i];
        ufp[s] |= fp[i];
      }
    }
  std::ostringstream o;
  o << "// Generated burn kernel: N = " << N << " species, R = " << R
    << " reactions, " << lpc << " lane(s) per cell.\n";
  o << "#include \"burn_gen_body.h\"\nnamespace bng {\nstruct GenNet {\n";
  o << "  static constexpr int N = " << N << ", R = " << R << ", n = " << n << ";\n";
  o << "  static constexpr int NS = " << NS << ", RB = " << (R + 7) / 8 * 8 << ";\n";
  o << "  static constexpr unsigned long long fpat[n] = {";
  for (int i = 0; i < n; ++i) o << (i ? ", " : "") << "0x" << std::hex << fp[i] << std::dec << "ull";
  o << "};\n  static constexpr unsigned long long ufill[NS] = {";
  for (int s = 0; s < NS; ++s) o << (s ? ", " : "") << "0x" << std::hex << ufp[s] << std::dec << "ull";
  o << "};\n";
  // the heat row's quotients by c_v: q = x (1/c_v), then Markstein's
  // correction step, which gives the correctly rounded x / c_v wherever that
  // is a normal number (a non-finite x gives a non-finite result, which every
  // caller treats alike)
  o << "  static constexpr double cv = " << hexd(d.c_v) << ", icv = " << hexd(1.0 / d.c_v) << ";\n";
  o << "  __device__ __forceinline__ static double div_cv(double x) {\n"
       "    const double q = x * icv;\n    return fma(fma(-q, cv, x), icv, q);\n  }\n";
  const int RT = (R + lpc - 1) / lpc;  // rate exponentials per lane
  if (lpc > 1) {
    // the rate coefficients as a table that the kernel copies into the LDS:
    // the lanes of a cell evaluate different reactions' exponentials (lane h
    // takes reactions t * lpc + h), each reading its own coefficients;
    // padding rows are zero
    o << "  static constexpr int RT = " << RT << ";\n";
    o << "  static constexpr double ctab[" << RT * lpc * 8 << "] = {";
    for (int r = 0; r < RT * lpc; ++r)
      for (int j = 0; j < 8; ++j)
        o << ((r || j) ? ", " : "") << ((r < R && j < 7) ? hexd(d.coef[7 * r + j]) : std::string("0.0"));
    o << "};\n";
  }
  o << "  static constexpr long long HOST_LDS = " << gen_lds_bytes(d, lpc) << ";\n";

  // T powers, as in the rate definition
  const char *tpow =
      "    const double T = y[N];\n"
      "    const double t13 = cbrt(T);\n"
      "    const double tm13 = 1.0 / t13;\n"
      "    const double t53 = T * t13 * t13;\n"
      "    const double lnT = bn::bn_log(T);\n"
      "    const double tinv = 1.0 / T;\n";
  auto lam_expr = [&](int r) {
    const double *a = d.coef.data() + 7 * r;
    std::ostringstream e;
    e << "exp(fma(" << hexd(a[6]) << ", lnT, fma(" << hexd(a[5]) << ", t53, fma(" << hexd(a[4])
      << ", T, fma(" << hexd(a[3]) << ", t13, fma(" << hexd(a[2]) << ", tm13, fma(" << hexd(a[1])
      << ", tinv, " << hexd(a[0]) << "))))))) * em[" << r << "]";
    return e.str();
  };
  // the exponentials l<r> of every reaction, in every lane of the cell
  // (with several lanes per cell each lane evaluates its share, read from
  // the LDS table at em + RB, and broadcasts it)
  auto emit_lams = [&](const char *ind) {
    if (lpc == 1) {
      for (int r = 0; r < R; ++r) o << ind << "const double l" << r << " = " << lam_expr(r) << ";\n";
      return;
    }
    o << ind << "double lo[RT];\n" << ind << "{\n"
      << ind << "  const double *ct = em + RB + h * 8;\n"
      << ind << "#pragma unroll\n" << ind << "  for (int t = 0; t < RT; ++t) {\n"
      << ind << "    const double2 *c = (const double2 *)(ct + t * " << lpc * 8 << ");\n"
      << ind << "    const double2 c01 = c[0], c23 = c[1], c45 = c[2], c6 = c[3];\n"
      << ind << "    lo[t] = exp(fma(c6.x, lnT, fma(c45.y, t53, fma(c45.x, T, fma(c23.y, t13, "
                "fma(c23.x, tm13, fma(c01.y, tinv, c01.x))))))) * em[t * " << lpc << " + h];\n"
      << ind << "  }\n" << ind << "}\n";
    for (int r = 0; r < R; ++r)
      o << ind << "const double l" << r << " = Grp<" << lpc << ">::template bcast<" << r % lpc
        << ">(lo[" << r / lpc << "]);\n";
  };
  // prefactor lambda / prod m! rho^(n_r - 1)
  auto pre_expr = [&](int r) {
    int nr = 0;
    const double f = inv_fact(d, r, &nr);
    std::string e = "l" + std::to_string(r);
    if (f != 1.0) e = "(" + e + " * " + hexd(f) + ")";
    for (int i = 1; i < nr; ++i) e = "(" + e + " * rho)";
    return e;
  };
  auto rate_expr = [&](int r) {
    std::string e = "p" + std::to_string(r);
    for (int a = 0; a < 3; ++a)
      if (d.reac[3 * r + a] >= 0) e = "(" + e + " * y[" + std::to_string(d.reac[3 * r + a]) + "])";
    return e;
  };
  auto own = [&](const std::string &dst, int s, const std::vector<std::string> &vals) {
    // vals[hh]: value of row s * lpc + hh ("" = zero)
    std::string v0 = vals[0].empty() ? "0.0" : vals[0];
    if (lpc == 1) return dst + " = " + v0 + ";\n";
    std::string v1 = vals[1].empty() ? "0.0" : vals[1];
    return dst + " = h ? " + v1 + " : " + v0 + ";\n";
  };

  // ---- right-hand side
  o << "  __device__ __forceinline__ static void rhs(const double (&y)[n], double rho, "
       "const double *em, int h, double (&F)[NS]) {\n"
       "#pragma clang fp contract(off)\n";
  o << tpow;
  // every sum starts at 0 and takes its terms in ascending reaction order,
  // each rate as soon as it is formed
  emit_lams("    ");
  o << "    double e = 0.0";
  for (int i = 0; i < N; ++i) o << ", f" << i << " = 0.0";
  o << ";\n";
  for (int r = 0; r < R; ++r) {
    o << "    {\n      const double p" << r << " = " << pre_expr(r) << ";\n";
    o << "      const double r" << r << " = " << rate_expr(r) << ";\n";
    for (int i = 0; i < N; ++i) {
      const int v = nu_of(d, i, r);
      if (v) o << "      f" << i << " = f" << i << " + " << wterm(v, "r" + std::to_string(r)) << ";\n";
    }
    o << "      e = e + " << hexd(d.q[r]) << " * r" << r << ";\n    }\n";
  }
  std::vector<std::string> fexpr(n);
  for (int i = 0; i < N; ++i) fexpr[i] = "f" + std::to_string(i);
  o << "    const double f" << N << " = div_cv(e);\n";
  fexpr[N] = "f" + std::to_string(N);
  for (int s = 0; s < NS; ++s) {
    std::vector<std::string> vals(lpc);
    for (int hh = 0; hh < lpc; ++hh)
      if (s * lpc + hh < n) vals[hh] = fexpr[s * lpc + hh];
    o << "    " << own("F[" + std::to_string(s) + "]", s, vals);
  }
  o << "  }\n";

  // compact index of the own Jacobian entries (union over the slot's rows)
  std::vector<std::vector<int>> eidx(NS, std::vector<int>(n, -1));
  int ne = 0;
  for (int s = 0; s < NS; ++s)
    for (int j = 0; j < n; ++j)
      if ((ujp[s] >> j) & 1ull) eidx[s][j] = ne++;
  o << "  static constexpr int NE = " << ne << ";\n";
  auto diag = [&](int s, int j) {
    // (I)_{comp(s), j}
    const int lo = s * lpc, hi = s * lpc + lpc - 1;
    if (j < lo || j > hi) return std::string("0.0");
    if (lpc == 1) return std::string("1.0");
    return std::string("(h == ") + std::to_string(j - lo) + " ? 1.0 : 0.0)";
  };

  // ---- Jacobian into the workspace and the Newton matrix
  o << "  __device__ __forceinline__ static void jac_m(const double (&y)[n], double rho, "
       "const double *em, int h, double cc, double (&M)[NS][n], gptr jb, long long NL, "
       "int &jbad) {\n"
       "#pragma clang fp contract(off)\n";
  o << tpow;
  emit_lams("    ");
  for (int r = 0; r < R; ++r) o << "    const double p" << r << " = " << pre_expr(r) << ";\n";
  // One column at a time: its terms (one per reactant slot holding the
  // species, the product of the other slots; the temperature column last,
  // dR/dT = R d ln lambda / dT), then the own entries of that column.
  o << "    int bad = 0;\n";
  auto emit_column = [&](int j, const std::vector<std::string> &Jc) {
    for (int s2 = 0; s2 < NS; ++s2) {
      if (eidx[s2][j] < 0) continue;
      const std::string ms = "M[" + std::to_string(s2) + "][" + std::to_string(j) + "]";
      std::vector<std::string> vals(lpc);
      for (int hh = 0; hh < lpc; ++hh)
        if (s2 * lpc + hh < n) vals[hh] = Jc[s2 * lpc + hh];
      o << "      {\n        double jv;\n        " << own("jv", s2, vals);
      o << "        if (!__builtin_isfinite(jv)) bad = 1;\n";
      o << "        jb[" << eidx[s2][j] << "ll * NL] = jv;\n";
      o << "        " << ms << " = " << diag(s2, j) << " - cc * jv;\n      }\n";
    }
  };
  for (int j = 0; j < N; ++j) {
    std::vector<std::string> Jc(n);
    o << "    {\n";
    for (int r = 0; r < R; ++r)
      for (int a = 0; a < 3; ++a) {
        if (d.reac[3 * r + a] != j) continue;
        std::string x = "p" + std::to_string(r);
        for (int b = 0; b < 3; ++b)
          if (b != a && d.reac[3 * r + b] >= 0)
            x = "(" + x + " * y[" + std::to_string(d.reac[3 * r + b]) + "])";
        const std::string nm = "x" + std::to_string(r) + "_" + std::to_string(a);
        o << "      const double " << nm << " = " << x << ";\n";
        for (int i = 0; i < N; ++i) {
          const int v = nu_of(d, i, r);
          if (!v) continue;
          std::string &e = Jc[i];
          if (e.empty()) e = "0.0";
          e = "(" + e + " + " + wterm(v, nm) + ")";
        }
        std::string &e = Jc[N];
        if (e.empty()) e = "0.0";
        e = "(" + e + " + div_cv(" + hexd(d.q[r]) + " * " + nm + "))";
      }
    emit_column(j, Jc);
    o << "    }\n";
  }
  {
    std::vector<std::string> Jc(n);
    o << "    {\n";
    for (int r = 0; r < R; ++r) {
      const double *a = d.coef.data() + 7 * r;
      const double c2 = (1.0 / 3.0) * a[2], c3 = (1.0 / 3.0) * a[3], c5 = (5.0 / 3.0) * a[5];
      o << "      const double dT" << r << " = " << rate_expr(r) << " * ((((((" << hexd(-a[1])
        << " * tinv * tinv - " << hexd(c2) << " * tm13 * tinv) + " << hexd(c3)
        << " * t13 * tinv) + " << hexd(a[4]) << ") + " << hexd(c5) << " * t13 * t13) + "
        << hexd(a[6]) << " * tinv));\n";
      for (int i = 0; i < N; ++i) {
        const int v = nu_of(d, i, r);
        if (!v) continue;
        std::string &e = Jc[i];
        if (e.empty()) e = "0.0";
        e = "(" + e + " + " + wterm(v, "dT" + std::to_string(r)) + ")";
      }
      std::string &e = Jc[N];
      if (e.empty()) e = "0.0";
      e = "(" + e + " + div_cv(" + hexd(d.q[r]) + " * dT" + std::to_string(r) + "))";
    }
    emit_column(N, Jc);
    o << "    }\n";
  }
  // entries outside the Jacobian pattern of both rows: the identity's
  for (int s2 = 0; s2 < NS; ++s2)
    for (int j = 0; j < n; ++j)
      if (eidx[s2][j] < 0)
        o << "    M[" << s2 << "][" << j << "] = " << diag(s2, j) << ";\n";
  o << "    jbad = bad;\n  }\n";

  // ---- the Newton matrix from the workspace
  o << "  __device__ __forceinline__ static void load_m(int h, double cc, double (&M)[NS][n], "
       "gptr jb, long long NL) {\n"
       "#pragma clang fp contract(off)\n";
  for (int s = 0; s < NS; ++s)
    for (int j = 0; j < n; ++j) {
      const std::string ms = "M[" + std::to_string(s) + "][" + std::to_string(j) + "]";
      if (eidx[s][j] < 0)
        o << "    " << ms << " = " << diag(s, j) << ";\n";
      else
        o << "    " << ms << " = " << diag(s, j) << " - cc * jb[" << eidx[s][j] << "ll * NL];\n";
    }
  o << "  }\n};\n}  // namespace bng\n\n";
  o << "extern \"C\" __global__ void __launch_bounds__(256) "
       "__attribute__((amdgpu_waves_per_eu(1, 1))) bn_gen_burn(bng::GenArgs a) {\n"
       "  bng::burn_kernel_body<bng::GenNet, "
    << lpc << ">(a);\n}\n";
  return o.str();
}

int gen_entries(const GenDesc &d, int lpc) {
  const int n = d.N + 1, NS = (n + lpc - 1) / lpc;
  std::vector<unsigned long long> jp;
  jac_pattern(d, &jp);
  int ne = 0;
  for (int s = 0; s < NS; ++s) {
    unsigned long long u = 0;
    for (int hh = 0; hh < lpc; ++hh)
      if (s * lpc + hh < n) u |= jp[s * lpc + hh];
    ne += __builtin_popcountll(u);
  }
  return ne;
}

size_t gen_lds_bytes(const GenDesc &d, int lpc) {
  const int n = d.N + 1, NS = (n + lpc - 1) / lpc;
  // the rate multipliers (rounded up to 8), the coefficient table when the
  // lanes of a cell split the rates, then four waves of [rows][NS][64]: the
  // history (7 rows), psi and the reciprocal scales, and the Newton
  // correction and reciprocal pivots when they fit in the LDS of a compute
  // unit; the head ends with the reciprocals 1/j of j = 0..7.  The generated
  // source carries this size and the kernel checks at compile time that its
  // own layout needs exactly this much.
  const size_t head = (size_t)(d.R + 7) / 8 * 8 + (lpc > 1 ? (size_t)(d.R + lpc - 1) / lpc * lpc * 8 : 0) + 8;
  const size_t full = 8 * (head + (size_t)4 * 11 * NS * 64);
  return full <= 160 * 1024 ? full : 8 * (head + (size_t)4 * 9 * NS * 64);
}

const std::vector<std::string> &gen_options() {
  static const std::vector<std::string> opts = {
      "--offload-arch=gfx950", "-O3", "-std=c++20",
      // no packed-FP32 instructions (all arithmetic here is FP64)
      "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  return opts;
}

uint64_t gen_key(const std::string &src) {
  uint64_t hsh = 1469598103934665603ull;  // FNV-1a 64
  auto mix = [&](const char *p, size_t len) {
    for (size_t i = 0; i < len; ++i) {
      hsh ^= (unsigned char)p[i];
      hsh *= 1099511628211ull;
    }
  };
  mix(src.data(), src.size());
  mix(BNG_BODY_H, sizeof(BNG_BODY_H));
  mix(BNG_ARGS_H, sizeof(BNG_ARGS_H));
  mix(BNG_MATH_H, sizeof(BNG_MATH_H));
  for (const std::string &s : gen_options()) mix(s.data(), s.size() + 1);
  int major = 0, minor = 0;
  if (hiprtcVersion(&major, &minor) == HIPRTC_SUCCESS) {
    mix(reinterpret_cast<const char *>(&major), sizeof major);
    mix(reinterpret_cast<const char *>(&minor), sizeof minor);
  }
  return hsh;
}

std::string gen_cache_path(const std::string &dir, uint64_t key) {
  char buf[32];
  std::snprintf(buf, sizeof buf, "bng_%016llx.co", (unsigned long long)key);
  return dir + "/" + buf;
}

bool gen_cache_read(const std::string &path, std::vector<char> *code) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  code->assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
  return !code->empty();
}

void gen_cache_write(const std::string &dir, const std::string &path, const std::vector<char> &code) {
  ::mkdir(dir.c_str(), 0755);  // one level; an existing directory is fine
  const std::string tmp = path + ".tmp" + std::to_string((long long)::getpid());
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(code.data(), (std::streamsize)code.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), path.c_str());
}

int gen_compile(const std::string &src, std::vector<char> *code, std::string *log) {
  hiprtcProgram prog;
  const char *hdrs[3] = {BNG_BODY_H, BNG_ARGS_H, BNG_MATH_H};
  const char *names[3] = {"burn_gen_body.h", "burn_gen_args.h", "bn_math.h"};
  if (hiprtcCreateProgram(&prog, src.c_str(), "bn_gen_burn.hip", 3, hdrs, names) != HIPRTC_SUCCESS) {
    *log = "hiprtcCreateProgram failed";
    return -1;
  }
  std::vector<const char *> opts;
  for (const std::string &s : gen_options()) opts.push_back(s.c_str());
  const hiprtcResult rc = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  size_t ls = 0;
  if (hiprtcGetProgramLogSize(prog, &ls) == HIPRTC_SUCCESS && ls > 1) {
    std::string l(ls, '\0');
    if (hiprtcGetProgramLog(prog, &l[0]) == HIPRTC_SUCCESS) *log = l;
  }
  if (rc != HIPRTC_SUCCESS) {
    (void)hiprtcDestroyProgram(&prog);
    if (log->empty()) *log = hiprtcGetErrorString(rc);
    return -1;
  }
  size_t cs = 0;
  if (hiprtcGetCodeSize(prog, &cs) != HIPRTC_SUCCESS || cs == 0) {
    (void)hiprtcDestroyProgram(&prog);
    *log = "hiprtc returned no code";
    return -1;
  }
  code->resize(cs);
  const hiprtcResult rc2 = hiprtcGetCode(prog, code->data());
  (void)hiprtcDestroyProgram(&prog);
  if (rc2 != HIPRTC_SUCCESS) {
    *log = "hiprtcGetCode failed";
    return -1;
  }
  return 0;
}

int gen_build(const GenDesc &d, int lpc, const std::string &cache_dir, std::vector<char> *code,
              std::string *err) {
  const std::string src = gen_source(d, lpc);
  const uint64_t key = gen_key(src);
  std::string path;
  if (!cache_dir.empty()) {
    path = gen_cache_path(cache_dir, key);
    if (gen_cache_read(path, code)) return 0;
  }
  std::string log;
  if (gen_compile(src, code, &log) != 0) {
    *err = "compilation of the generated kernel failed: " + log;
    return -1;
  }
  if (!cache_dir.empty()) gen_cache_write(cache_dir, path, *code);
  return 0;
}

}  // namespace bn

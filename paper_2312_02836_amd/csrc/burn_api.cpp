// burn_api.cpp -- the C ABI declared in include/burn.h: network validation,
// device tables, argument checks and kernel dispatch.  No compute happens on
// the host: every step of the burn runs in the HIP kernels.

#include "burn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "burn_codegen.h"
#include "burn_gen_args.h"
#include "burn_internal.h"

// A network's generated kernel (bn_network_generate): the loaded module and
// the per-lane workspaces of its launch grid.
struct GenKernel {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int lpc = 0;              // lanes per cell
  size_t lds = 0;           // dynamic LDS per workgroup
  int grid = 0;             // workgroups (one per CU)
  long long n_lanes = 0;    // grid threads
  double *jws = nullptr;    // Jacobian rows [entries][n_lanes]
  double *lws = nullptr;    // pivoting scratch [n*n + 4n][n_lanes]
  unsigned long long *queue = nullptr;  // the unordered launch's counter
  // factorization batching of the wave (see the kernel's pass): a pass runs
  // once lu_batch cells want one or a cell has waited lu_wait iterations
  // (12 and 7 measured best on the 13/30 launch, about 18.1 ms against
  // 22.1 ms for a pass whenever any cell wants one; results are bitwise the
  // same)
  int lu_batch = 12, lu_wait = 7;
};

struct bn_network {
  int N = 0, R = 0, n = 0, nnz = 0;
  double c_v = 0.0;
  int device = 0;
  void *dev = nullptr;  // one allocation holding every table
  bn::NetTables tables{};
  // plain launch choice (0 = default for the system size)
  int L = 0, S = 0, block_waves = 0;
  double ms_per_cell = 0.0;  // measured by the autotuner (0 = unknown)
  // persistent launch choice (pW = 0: chosen per call from the plain choice
  // and the LDS footprint)
  int pL = 0, pS = 0, pW = 0, pbw = 0;
  bool screened = false;
  bn::GenDesc desc;         // host copy for code generation
  GenKernel *gen = nullptr;
  int body = BN_BODY_TABLE;
  // per-wave Jacobian areas of the persistent launches that factor in LDS
  // (systems above 16 components; see bn::BurnArgs::jws)
  void *jws = nullptr;
  size_t jws_bytes = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

// Net stoichiometric coefficient of species i in reaction r.
int nu_of(const bn_network_desc *d, int i, int r) {
  int v = 0;
  for (int s = 0; s < 3; ++s) {
    v += (d->products[3 * r + s] == i);
    v -= (d->reactants[3 * r + s] == i);
  }
  return v;
}

struct DeviceLimits {
  size_t lds_block = 64 * 1024;  // dynamic LDS per workgroup
  size_t lds_cu = 64 * 1024;     // LDS per compute unit
  int cus = 1;
};

int device_limits(int dev, DeviceLimits *out) {
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return fail(BN_EHIP, "hipDeviceGetAttribute(MaxSharedMemoryPerBlock) failed");
  out->lds_block = (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) !=
      hipSuccess)
    return fail(BN_EHIP, "hipDeviceGetAttribute(MaxSharedMemoryPerMultiprocessor) failed");
  out->lds_cu = (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(BN_EHIP, "hipDeviceGetAttribute(MultiprocessorCount) failed");
  out->cus = v > 0 ? v : 1;
  return BN_SUCCESS;
}

bool plain_shape(int L, int S) {
  for (const bn::ShapeLS &sh : bn::PLAIN_SHAPES)
    if (sh.L == L && sh.S == S) return true;
  return false;
}

// waves per SIMD a plain shape is compiled for
int plain_waves(int L, int S) {
  for (const bn::ShapeLS &sh : bn::PLAIN_SHAPES)
    if (sh.L == L && sh.S == S) return sh.W;
  return 1;
}

// index of (L, S) in MULTI_SHAPES_2 (the two-waves-per-SIMD set used by the
// persistent kernel and the recording / source / screened kernels), or -1
int multi_shape_index(int L, int S) {
  for (int i = 0; i < bn::N_MULTI_SHAPES; ++i)
    if (bn::MULTI_SHAPES_2[i].L == L && bn::MULTI_SHAPES_2[i].S == S) return i;
  return -1;
}

int multi1_shape_index(int L, int S) {
  for (int i = 0; i < bn::N_MULTI_SHAPES; ++i)
    if (bn::MULTI_SHAPES_1[i].L == L && bn::MULTI_SHAPES_1[i].S == S) return i;
  return -1;
}

// Default shape for a system of size n (before any tuning): the narrowest
// group whose padded size holds the system, at two waves per SIMD.
void default_shape(int n, int *L, int *S) {
  if (n <= 4) { *L = 4; *S = 1; }
  else if (n <= 8) { *L = 8; *S = 1; }
  else if (n <= 16) { *L = 16; *S = 1; }
  else if (n <= 32) { *L = 32; *S = 1; }
  else { *L = 64; *S = 1; }
}

// Default within MULTI_SHAPES_2.
void default_multi_shape(int n, int *L, int *S) {
  if (n <= 8) { *L = 8; *S = 1; }
  else if (n <= 16) { *L = 16; *S = 1; }
  else if (n <= 32) { *L = 32; *S = 1; }
  else { *L = 64; *S = 1; }
}

// Default within MULTI_SHAPES_1.
void default_multi1_shape(int n, int *L, int *S) {
  if (n <= 16) { *L = 4; *S = 4; }
  else if (n <= 32) { *L = 16; *S = 2; }
  else { *L = 64; *S = 1; }
}

// Shape for a plain launch: an explicit lanes hint picks the smallest
// padded size with that L; else the network's choice; else the default.
bool pick_shape(const bn_network *net, int lanes_hint, int *L, int *S) {
  if (lanes_hint) {
    for (const bn::ShapeLS &sh : bn::PLAIN_SHAPES)
      if (sh.L == lanes_hint && sh.L * sh.S >= net->n) {
        *L = sh.L;
        *S = sh.S;
        return true;
      }
    return false;
  }
  if (net->L) {
    *L = net->L;
    *S = net->S;
    return true;
  }
  default_shape(net->n, L, S);
  return true;
}

size_t lds_bytes(int R, int L, int S, int n, int bw) {
  return bn::table_lds_bytes(R) + (size_t)bw * bn::wave_lds_bytes(L, S, n);
}

void fill_desc(const bn_network_desc *d, bn::GenDesc *g) {
  g->N = d->n_species;
  g->R = d->n_reactions;
  g->mass.assign(d->mass, d->mass + g->N);
  g->reac.assign(d->reactants, d->reactants + 3 * g->R);
  g->prod.assign(d->products, d->products + 3 * g->R);
  g->coef.assign(d->coef, d->coef + 7 * g->R);
  g->q.assign(d->q, d->q + g->R);
  g->c_v = d->c_v;
}

void free_gen(GenKernel *g) {
  if (!g) return;
  if (g->mod) (void)hipModuleUnload(g->mod);
  if (g->jws) (void)hipFree(g->jws);
  if (g->lws) (void)hipFree(g->lws);
  if (g->queue) (void)hipFree(g->queue);
  delete g;
}

// lanes per cell of the generated body for a system of n components (0:
// none supported), or check an explicit choice
int gen_lanes(int n, int want) {
  if (want == 1) return n <= bn::GEN_MAX_N1 ? 1 : 0;
  if (want == 2) return n <= bn::GEN_MAX_N2 ? 2 : 0;
  if (want != 0) return 0;
  if (n <= bn::GEN_MAX_N1) return 1;
  if (n <= bn::GEN_MAX_N2) return 2;
  return 0;
}

// Launch the generated kernel over the cells of a (for an ordered launch:
// staged) batch; parts = the XCD part counters, or null for the kernel's
// own queue counter (reset here by a kernel).
hipError_t launch_gen(const bn_network *net, const bn::BurnArgs &a, unsigned long long *queue,
                      hipStream_t st) {
  const GenKernel &g = *net->gen;
  bng::GenArgs ga{};
  ga.Y = a.Y;
  ga.T = a.T;
  ga.rho = a.rho;
  ga.status = a.status;
  ga.counters = a.counters;
  ga.log_mult = a.log_mult;
  ga.jws = g.jws;
  ga.lws = g.lws;
  ga.queue = queue;
  ga.parts = a.parts;
  ga.n_cells = a.n_cells;
  ga.n_lanes = g.n_lanes;
  ga.t_end = a.t_end;
  ga.rtol = a.rtol;
  ga.atol = a.atol;
  ga.max_steps = a.max_steps;
  ga.lu_batch = g.lu_batch;
  ga.lu_wait = g.lu_wait;
  if (!a.parts) {
    const hipError_t e = bn::launch_zero(queue, 1, st);
    if (e != hipSuccess) return e;
  }
  void *params[] = {&ga};
  return hipModuleLaunchKernel(g.fn, (unsigned)g.grid, 1, 1, 256, 1, 1, (unsigned)g.lds, st, params,
                               nullptr);
}

int check_tol(double dt, double rtol, double atol) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BN_EINVAL, "dt must be positive and finite");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(BN_EINVAL, "rtol must be positive");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(BN_EINVAL, "atol must be >= 0");
  return BN_SUCCESS;
}

}  // namespace

extern "C" {

const char *bn_last_error(void) { return g_err.c_str(); }

const char *bn_version(void) { return "mi355x-burn 0.1 (gfx950, FP64 BDF)"; }

int bn_network_create(const bn_network_desc *d, bn_network **out) {
  g_err.clear();
  if (!d || !out) return fail(BN_EINVAL, "null argument");
  *out = nullptr;
  const int N = d->n_species, R = d->n_reactions;
  if (N < 1 || R < 1) return fail(BN_EINVAL, "need n_species >= 1 and n_reactions >= 1");
  if (N + 1 > BN_MAX_SYSTEM)
    return fail(BN_EUNSUPPORTED, "n_species + 1 exceeds BN_MAX_SYSTEM");
  if (R > BN_MAX_REACTIONS) return fail(BN_EUNSUPPORTED, "n_reactions exceeds BN_MAX_REACTIONS");
  if (!d->mass || !d->reactants || !d->products || !d->coef || !d->q)
    return fail(BN_EINVAL, "null table pointer in bn_network_desc");
  if (!(d->c_v > 0.0) || !std::isfinite(d->c_v)) return fail(BN_EINVAL, "c_v must be positive");
  for (int i = 0; i < N; ++i)
    if (d->mass[i] < 1) return fail(BN_EINVAL, "mass numbers must be >= 1");
  for (int r = 0; r < R; ++r) {
    int used = 0;
    long long ma = 0, mb = 0;
    for (int s = 0; s < 3; ++s) {
      const int a = d->reactants[3 * r + s], b = d->products[3 * r + s];
      if (a < -1 || a >= N || b < -1 || b >= N)
        return fail(BN_EINVAL, "species index out of range in reaction " + std::to_string(r));
      if (a >= 0) {
        ++used;
        ma += d->mass[a];
      }
      if (b >= 0) mb += d->mass[b];
    }
    if (!used) return fail(BN_EINVAL, "reaction " + std::to_string(r) + " has no reactant");
    if (ma != mb)
      return fail(BN_EINVAL, "reaction " + std::to_string(r) + " does not conserve mass number");
    for (int c = 0; c < 7; ++c)
      if (!std::isfinite(d->coef[7 * r + c])) return fail(BN_EINVAL, "non-finite rate coefficient");
    if (!std::isfinite(d->q[r])) return fail(BN_EINVAL, "non-finite heat q");
    if (d->screen && !std::isfinite(d->screen[r]))
      return fail(BN_EINVAL, "non-finite screening strength");
  }

  // Host copies of the tables.
  std::vector<double> rtab((size_t)R * bn::RTAB), q(d->q, d->q + R);
  std::vector<int> rsp(4 * (size_t)R);
  for (int r = 0; r < R; ++r) {
    for (int c = 0; c < 7; ++c) rtab[(size_t)r * bn::RTAB + c] = d->coef[7 * r + c];
    // 1 / prod over distinct reactant species of (multiplicity)!
    const int *s = d->reactants + 3 * r;
    double f = 1.0;
    int nr = 0;
    for (int i = 0; i < 3; ++i) {
      if (s[i] < 0) continue;
      ++nr;
      bool first = true;
      for (int j = 0; j < i; ++j)
        if (s[j] == s[i]) first = false;
      if (!first) continue;
      int m = 0;
      for (int j = 0; j < 3; ++j) m += (s[j] == s[i]);
      for (int j = 2; j <= m; ++j) f *= (double)j;
    }
    rtab[(size_t)r * bn::RTAB + 7] = 1.0 / f;
    for (int i = 0; i < 3; ++i) rsp[4 * r + i] = s[i];
    rsp[4 * r + 3] = nr;
  }
  std::vector<int> row_off(N + 1), row_r;
  std::vector<double> row_w;
  for (int i = 0; i < N; ++i) {
    row_off[i] = (int)row_r.size();
    for (int r = 0; r < R; ++r) {
      const int v = nu_of(d, i, r);
      if (v) {
        row_r.push_back(r);
        row_w.push_back((double)v);
      }
    }
  }
  row_off[N] = (int)row_r.size();
  const int nnz = (int)row_r.size();
  // reactant-slot lists per species column, and the dense nu table
  std::vector<int> col_off(N + 1), col_ent;
  for (int j = 0; j < N; ++j) {
    col_off[j] = (int)col_ent.size();
    for (int r = 0; r < R; ++r)
      for (int a = 0; a < 3; ++a)
        if (d->reactants[3 * r + a] == j) col_ent.push_back((r << 2) | a);
  }
  col_off[N] = (int)col_ent.size();
  const int nsl = (int)col_ent.size();
  std::vector<signed char> nu8((size_t)N * R);
  for (int i = 0; i < N; ++i)
    for (int r = 0; r < R; ++r) nu8[(size_t)i * R + r] = (signed char)nu_of(d, i, r);
  // per reaction: the species it changes and by how much (at most 6)
  std::vector<int> rout(8 * (size_t)R, 0);
  int max_ent = 0;
  for (int r = 0; r < R; ++r) {
    int c = 0;
    for (int i = 0; i < N; ++i) {
      const int v = nu_of(d, i, r);
      if (v) rout[8 * r + 1 + c++] = (i << 8) | (v & 0xff);
    }
    rout[8 * r] = c;
    if (c > max_ent) max_ent = c;
    // entries past the count: coefficient 0 on the first listed species
    for (int e = c; e < 6; ++e) rout[8 * r + 1 + e] = c ? (rout[8 * r + 1] & ~0xff) : 0;
  }

  auto *net = new bn_network();
  net->N = N;
  net->R = R;
  net->n = N + 1;
  net->nnz = nnz;
  net->c_v = d->c_v;
  if (hipGetDevice(&net->device) != hipSuccess) {
    delete net;
    return fail(BN_EHIP, "hipGetDevice failed");
  }
  std::vector<double> scr, wsq(N);
  if (d->screen) scr.assign(d->screen, d->screen + R);
  for (int i = 0; i < N; ++i) wsq[i] = (double)d->mass[i] * (double)d->mass[i];
  // Layout of the device block: doubles first, then ints.
  const size_t nd = rtab.size() + q.size() + row_w.size() + scr.size() + wsq.size();
  const size_t ni = rsp.size() + row_off.size() + row_r.size() + col_off.size() + col_ent.size() +
                    rout.size();
  const size_t bytes = nd * 8 + ni * 4 + nu8.size() + 16;
  if (hipMalloc(&net->dev, bytes) != hipSuccess) {
    delete net;
    (void)hipGetLastError();
    return fail(BN_ENOMEM, "hipMalloc of the network tables failed");
  }
  std::vector<char> host(bytes, 0);
  size_t off = 0;
  auto put = [&](const void *src, size_t nbytes) {
    std::memcpy(host.data() + off, src, nbytes);
    const size_t at = off;
    off += nbytes;
    return at;
  };
  const size_t o_rtab = put(rtab.data(), rtab.size() * 8);
  const size_t o_q = put(q.data(), q.size() * 8);
  const size_t o_roww = put(row_w.data(), row_w.size() * 8);
  const size_t o_scr = put(scr.data(), scr.size() * 8);
  const size_t o_wsq = put(wsq.data(), wsq.size() * 8);
  const size_t o_rsp = put(rsp.data(), rsp.size() * 4);
  const size_t o_rowoff = put(row_off.data(), row_off.size() * 4);
  const size_t o_rowr = put(row_r.data(), row_r.size() * 4);
  const size_t o_coloff = put(col_off.data(), col_off.size() * 4);
  const size_t o_colent = put(col_ent.data(), col_ent.size() * 4);
  const size_t o_rout = put(rout.data(), rout.size() * 4);
  const size_t o_nu8 = put(nu8.data(), nu8.size());
  if (hipMemcpy(net->dev, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(net->dev);
    delete net;
    return fail(BN_EHIP, "hipMemcpy of the network tables failed");
  }
  char *base = static_cast<char *>(net->dev);
  bn::NetTables &t = net->tables;
  t.N = N;
  t.R = R;
  t.n = N + 1;
  t.nnz = nnz;
  t.inv_cv = 1.0 / d->c_v;
  t.rtab = reinterpret_cast<const double *>(base + o_rtab);
  t.q = reinterpret_cast<const double *>(base + o_q);
  t.row_w = reinterpret_cast<const double *>(base + o_roww);
  t.rsp = reinterpret_cast<const int *>(base + o_rsp);
  t.row_off = reinterpret_cast<const int *>(base + o_rowoff);
  t.row_r = reinterpret_cast<const int *>(base + o_rowr);
  t.nsl = nsl;
  t.max_ent = max_ent;
  t.col_off = reinterpret_cast<const int *>(base + o_coloff);
  t.col_ent = reinterpret_cast<const int *>(base + o_colent);
  t.nu8 = reinterpret_cast<const signed char *>(base + o_nu8);
  t.rout = reinterpret_cast<const int *>(base + o_rout);
  t.screen = d->screen ? reinterpret_cast<const double *>(base + o_scr) : nullptr;
  t.wsq = reinterpret_cast<const double *>(base + o_wsq);
  net->screened = d->screen != nullptr;
  fill_desc(d, &net->desc);
  // Room for the largest persistent grid of a shape that factors in LDS:
  // at most eight waves per compute unit, each holding 64 / L cells of
  // n^2 doubles (16 n^2 per unit when n <= 32 admits the 32-row shapes,
  // else 8 n^2).  Without it (allocation failed) every pass assembles J.
  if (!net->screened && t.n > 16) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, net->device) ==
            hipSuccess &&
        cus > 0) {
      const size_t jb = (size_t)cus * (t.n <= 32 ? 16 : 8) * (size_t)t.n * (size_t)t.n * 8;
      if (hipMalloc(&net->jws, jb) == hipSuccess) {
        net->jws_bytes = jb;
      } else {
        net->jws = nullptr;
        (void)hipGetLastError();
      }
    }
  }
  *out = net;
  return BN_SUCCESS;
}

void bn_network_destroy(bn_network *net) {
  if (!net) return;
  if (net->dev) (void)hipFree(net->dev);
  if (net->jws) (void)hipFree(net->jws);
  free_gen(net->gen);
  delete net;
}

int bn_network_n_species(const bn_network *net) { return net ? net->N : -1; }
int bn_network_n_reactions(const bn_network *net) { return net ? net->R : -1; }

int burn_batch_ex(const bn_network *net, int64_t n_cells, double *state, const double *rho,
                  double *T, double dt, double rtol, double atol, const double *log_mult,
                  int32_t *status, int32_t *counters, const bn_burn_opts *opts, void *stream) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (n_cells < 0) return fail(BN_EINVAL, "n_cells < 0");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  bn_burn_opts o{};
  if (opts) o = *opts;
  if (o.max_steps <= 0) o.max_steps = 100000;
  if (o.lanes_per_cell != 0 && o.lanes_per_cell != 4 && o.lanes_per_cell != 8 &&
      o.lanes_per_cell != 16 && o.lanes_per_cell != 32 && o.lanes_per_cell != 64)
    return fail(BN_EINVAL, "lanes_per_cell must be 0, 4, 8, 16, 32 or 64");
  if (o.block_waves < 0 || o.block_waves > 4) return fail(BN_EINVAL, "block_waves must be 0..4");
  if (n_cells == 0) return BN_SUCCESS;
  if (!state || !rho || !T) return fail(BN_EINVAL, "null state, rho or T");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;

  int L = 0, S = 0;
  if (!pick_shape(net, o.lanes_per_cell, &L, &S))
    return fail(BN_EUNSUPPORTED, "no kernel shape for this system size and lanes_per_cell");

  bn::BurnArgs a{};
  a.net = net->tables;
  a.n_cells = n_cells;
  a.Y = state;
  a.rho = rho;
  a.T = T;
  a.log_mult = log_mult;
  a.status = status;
  a.counters = counters;
  a.t_end = dt;
  a.rtol = rtol;
  a.atol = atol;
  a.max_steps = o.max_steps;

  if (net->body == BN_BODY_GENERATED && !o.lanes_per_cell) {
    const hipError_t e = launch_gen(net, a, net->gen->queue, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
      return fail(BN_EHIP, std::string("generated kernel launch failed: ") + hipGetErrorString(e));
    return BN_SUCCESS;
  }
  if (net->screened && multi_shape_index(L, S) < 0) {
    if (o.lanes_per_cell)
      return fail(BN_EUNSUPPORTED, "a screened network runs with 8, 16, 32 or 64 lanes per cell");
    default_multi_shape(net->n, &L, &S);
  }
  int bw = o.block_waves;
  if (bw == 0) {
    bw = (!o.lanes_per_cell && net->block_waves) ? net->block_waves
                                                  : (plain_waves(L, S) == 2 ? 1 : 2);
    while (bw > 1 && lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block) bw /= 2;
  }
  if (lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block)
    return fail(BN_EUNSUPPORTED, "network tables and working area exceed the LDS of a workgroup");
  const hipError_t e = net->screened
                           ? bn::launch_screen(a, L, S, bw, static_cast<hipStream_t>(stream))
                           : bn::launch_plain(a, L, S, bw, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BN_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BN_SUCCESS;
}

int burn_batch(const bn_network *net, int64_t n_cells, double *state, const double *rho,
               double *T, double dt, double rtol, double atol, const double *log_mult,
               int32_t *status, int32_t *counters, void *stream) {
  return burn_batch_ex(net, n_cells, state, rho, T, dt, rtol, atol, log_mult, status, counters,
                       nullptr, stream);
}


size_t burn_batch_multi_workspace_bytes(int32_t n_items) {
  if (n_items < 1) n_items = 1;
  return (((size_t)n_items * sizeof(unsigned long long)) + 255) / 256 * 256;
}

namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// Per item of an ordered launch, each region on a 256-byte boundary: the
// bucket counters, the per-XCD queue counters, h0 and the position of every
// cell, then the staged (position-ordered) state, T, rho, status and
// counters.
struct OrderLayout {
  size_t hist, parts, key, pos, Y, T, rho, status, counters, total;
};
OrderLayout order_layout(int64_t n, int N) {
  OrderLayout l{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  l.hist = take(2 * bn::ORDER_BUCKETS * sizeof(unsigned));
  l.parts = take(bn::XCD_PARTS * sizeof(unsigned long long));
  l.key = take((size_t)n * sizeof(float));
  l.pos = take((size_t)n * sizeof(int32_t));
  l.Y = take((size_t)n * N * sizeof(double));
  l.T = take((size_t)n * sizeof(double));
  l.rho = take((size_t)n * sizeof(double));
  l.status = take((size_t)n * sizeof(int32_t));
  l.counters = take((size_t)n * 8 * sizeof(int32_t));
  l.total = o;
  return l;
}
}  // namespace

size_t burn_batch_multi_order_workspace_bytes(int32_t n_items, const bn_batch_item *items) {
  size_t s = burn_batch_multi_workspace_bytes(n_items);
  if (!items) return s;
  for (int j = 0; j < n_items; ++j)
    if (items[j].n_cells > 0)
      s += order_layout(items[j].n_cells, items[j].net ? items[j].net->N : 0).total;
  return s;
}

}  // extern "C"

namespace {

// How an item runs in a persistent launch.
struct ItemLaunch {
  int W;      // waves per SIMD the kernel instance is compiled for (2 or 1)
  int L, S;   // shape
  int shape;  // index into MULTI_SHAPES_2 (W = 2) or MULTI_SHAPES_1 (W = 1)
  int bw;     // waves per workgroup
};

// The network's tuned persistent choice if it has one (bn_network_autotune_
// persistent); else two waves per SIMD with the network's plain choice when
// the two-wave kernel has that shape, or the default shape; else (a plain
// choice only the one-wave kernel has, or an LDS footprint that leaves fewer
// than six waves resident per CU at two) one wave per SIMD.  bw_opt
// overrides the waves per workgroup.
ItemLaunch item_launch(const bn_network *net, const DeviceLimits &lim, int bw_opt) {
  ItemLaunch r{};
  const int n = net->n;
  if (net->pW) {
    r.W = net->pW;
    r.L = net->pL;
    r.S = net->pS;
    r.bw = bw_opt ? bw_opt : net->pbw;
  } else {
    r.W = 2;
    r.L = net->L;
    r.S = net->S;
    if (r.L && multi_shape_index(r.L, r.S) < 0 && multi1_shape_index(r.L, r.S) >= 0) r.W = 1;
    if (r.W == 2 && (!r.L || multi_shape_index(r.L, r.S) < 0)) default_multi_shape(n, &r.L, &r.S);
    r.bw = bw_opt ? bw_opt : 4;
    if (r.W == 2) {
      const size_t tab = bn::table_lds_bytes(net->R), wave = bn::wave_lds_bytes(r.L, r.S, n);
      int bw = r.bw;
      while (bw > 1 && tab + (size_t)bw * wave > lim.lds_block) bw /= 2;
      const size_t lds = tab + (size_t)bw * wave;
      const size_t resident = std::min<size_t>(8 / bw, lim.lds_cu / lds) * bw;
      if (resident < 6) {
        r.W = 1;
        r.L = net->L;
        r.S = net->S;
      }
    }
    if (r.W == 1 && (!r.L || multi1_shape_index(r.L, r.S) < 0))
      default_multi1_shape(n, &r.L, &r.S);
  }
  r.shape = r.W == 2 ? multi_shape_index(r.L, r.S) : multi1_shape_index(r.L, r.S);
  return r;
}

// Side streams of a device for the launches of one multi-network call that
// run beside the first (default priority, non-blocking), with the events
// that fork them from and join them back to the caller's stream.  Created on
// first use and kept for the process.
struct SideStreams {
  hipStream_t s[BN_MAX_ITEMS] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t done[BN_MAX_ITEMS] = {};
  bool ok = false;
};
std::mutex g_side_mu;
SideStreams g_side[64];

// the side streams of device dev, or null if they cannot be made
SideStreams *side_streams(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  SideStreams &x = g_side[dev];
  if (x.ok) return &x;
  bool good = hipEventCreateWithFlags(&x.fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; good && i < BN_MAX_ITEMS; ++i)
    good = hipStreamCreateWithFlags(&x.s[i], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&x.done[i], hipEventDisableTiming) == hipSuccess;
  if (!good) {
    (void)hipGetLastError();
    return nullptr;  // the launches then run in order on the caller's stream
  }
  x.ok = true;
  return &x;
}

// burn_batch_multi with the workspace given (the caller's, or the library's
// static scratch for burn_batch_multi_noalloc).  Items that run at the same
// waves per SIMD share one persistent launch; a call with items of both
// kinds makes two launches, so that small networks are not held to the
// occupancy of large ones, and each generated network has a launch of its
// own.  With several launches, all but the first go to side streams forked
// from the caller's stream and joined back before the write-back, so that
// one launch's tail overlaps the others (allow_fork false, or a stream under
// graph capture: all in order on the caller's stream).
int multi_impl(int32_t n_items, const bn_batch_item *items, double dt, double rtol, double atol,
               const bn_burn_opts *opts, void *workspace, size_t workspace_bytes, void *stream,
               bool allow_fork) {
  if (n_items < 0 || n_items > BN_MAX_ITEMS)
    return fail(BN_EINVAL, "n_items must be 0..BN_MAX_ITEMS");
  if (n_items > 0 && !items) return fail(BN_EINVAL, "null items");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  bn_burn_opts o{};
  if (opts) o = *opts;
  if (o.max_steps <= 0) o.max_steps = 100000;
  if (o.lanes_per_cell != 0)
    return fail(BN_EINVAL, "lanes_per_cell must be 0 for burn_batch_multi");
  if (o.block_waves < 0 || o.block_waves > 4) return fail(BN_EINVAL, "block_waves must be 0..4");
  if (o.order_cells != 0 && o.order_cells != 1) return fail(BN_EINVAL, "order_cells must be 0 or 1");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;

  // validate and collect the non-empty items
  struct It {
    bn::BurnArgs a;
    ItemLaunch l;
    double cost;
    const bn_network *net;
  };
  std::vector<It> its;
  for (int j = 0; j < n_items; ++j) {
    const bn_batch_item &x = items[j];
    if (!x.net) return fail(BN_EINVAL, "null network in item " + std::to_string(j));
    if (x.net->device != dev) return fail(BN_EINVAL, "network was created on another device");
    if (x.n_cells < 0) return fail(BN_EINVAL, "n_cells < 0 in item " + std::to_string(j));
    if (x.net->screened)
      return fail(BN_EUNSUPPORTED, "screened networks are not supported by burn_batch_multi");
    if (x.n_cells == 0) continue;
    if (!x.state || !x.rho || !x.T)
      return fail(BN_EINVAL, "null state, rho or T in item " + std::to_string(j));
    It it{};
    it.net = x.net;
    it.l = item_launch(x.net, lim, o.block_waves);
    if (it.l.shape < 0) return fail(BN_EUNSUPPORTED, "no persistent kernel shape for item " +
                                                         std::to_string(j));
    bn::BurnArgs &a = it.a;
    a.net = x.net->tables;
    a.n_cells = x.n_cells;
    a.Y = x.state;
    a.rho = x.rho;
    a.T = x.T;
    a.log_mult = x.log_mult;
    a.status = x.status;
    a.counters = x.counters;
    a.t_end = dt;
    a.rtol = rtol;
    a.atol = atol;
    a.max_steps = o.max_steps;
    // cost per cell: measured if tuned, else a size model (LU ~ n^3, RHS ~ R)
    const double n = x.net->n;
    const double per = x.net->ms_per_cell > 0.0 ? x.net->ms_per_cell
                                                 : 1e-6 * (n * n * n + 40.0 * x.net->R);
    it.cost = per * (double)x.n_cells;
    its.push_back(it);
  }
  if (its.empty()) return BN_SUCCESS;
  const size_t need = o.order_cells ? burn_batch_multi_order_workspace_bytes(n_items, items)
                                    : burn_batch_multi_workspace_bytes(n_items);
  if (!workspace || workspace_bytes < need)
    return fail(BN_EINVAL, o.order_cells
                               ? "workspace missing or smaller than burn_batch_multi_order_workspace_bytes"
                               : "workspace missing or smaller than burn_batch_multi_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 8)
    return fail(BN_EINVAL, "workspace must be 8-byte aligned");
  // Items sorted: generated networks (each its own launch, enqueued after
  // the table-driven launches), then the two-wave class, then the one-wave
  // class; each class costliest network first (its cells then start first
  // and the tail is made of cheap ones).
  auto klass = [](const It &x) {
    return x.net->body == BN_BODY_GENERATED ? 0 : (x.l.W == 2 ? 1 : 2);
  };
  std::stable_sort(its.begin(), its.end(), [&](const It &x, const It &y) {
    if (klass(x) != klass(y)) return klass(x) < klass(y);
    return x.cost > y.cost;
  });

  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long *queue = static_cast<unsigned long long *>(workspace);
  hipError_t e = bn::launch_zero(queue, (int)its.size(), st);
  if (e != hipSuccess)
    return fail(BN_EHIP, std::string("counter reset launch failed: ") + hipGetErrorString(e));
  // ordered: each item's cells are staged in order of increasing initial
  // step size (stiffest first), burnt in that order and written back
  std::vector<bn::BurnArgs> orig(its.size()), staged(its.size());
  std::vector<int32_t *> posv(its.size(), nullptr);
  for (size_t j = 0; j < its.size(); ++j) staged[j] = orig[j] = its[j].a;
  if (o.order_cells) {
    char *p = static_cast<char *>(workspace) + burn_batch_multi_workspace_bytes(n_items);
    for (size_t j = 0; j < its.size(); ++j) {
      const bn::BurnArgs &a = orig[j];
      const OrderLayout l = order_layout(a.n_cells, a.net.N);
      unsigned *hist = reinterpret_cast<unsigned *>(p + l.hist);
      float *key = reinterpret_cast<float *>(p + l.key);
      int32_t *pos = reinterpret_cast<int32_t *>(p + l.pos);
      bn::BurnArgs s = a;
      s.Y = reinterpret_cast<double *>(p + l.Y);
      s.T = reinterpret_cast<double *>(p + l.T);
      s.rho = reinterpret_cast<const double *>(p + l.rho);
      s.status = a.status ? reinterpret_cast<int32_t *>(p + l.status) : nullptr;
      s.counters = a.counters ? reinterpret_cast<int32_t *>(p + l.counters) : nullptr;
      s.parts = reinterpret_cast<unsigned long long *>(p + l.parts);
      p += l.total;
      e = bn::launch_zero(reinterpret_cast<unsigned long long *>(hist), bn::ORDER_BUCKETS, st);
      if (e == hipSuccess) e = bn::launch_zero(s.parts, bn::XCD_PARTS, st);
      if (e == hipSuccess) e = bn::launch_order(a, key, pos, hist, lim.lds_block, st);
      if (e == hipSuccess) e = bn::launch_stage_in(a, s, pos, st);
      if (e != hipSuccess)
        return fail(BN_EHIP, std::string("queue order launch failed: ") + hipGetErrorString(e));
      posv[j] = pos;
      staged[j] = s;
    }
  }
  // the launches: the generated networks', then one persistent launch per
  // class (each a closure over its arguments, enqueued below)
  std::vector<std::function<hipError_t(hipStream_t)>> launches, gen_launches;
  size_t g0 = 0;
  for (; g0 < its.size() && klass(its[g0]) == 0; ++g0) {
    const bn_network *gnet = its[g0].net;
    const bn::BurnArgs ga = staged[g0];
    unsigned long long *gq = queue + g0;
    gen_launches.push_back([gnet, ga, gq](hipStream_t s) { return launch_gen(gnet, ga, gq, s); });
  }
  for (size_t c0 = g0; c0 < its.size();) {
    size_t c1 = c0;
    while (c1 < its.size() && klass(its[c1]) == klass(its[c0])) ++c1;
    const int W = its[c0].l.W;
    bn::MultiArgs m{};
    m.n_items = (int)(c1 - c0);
    size_t tabd = 0, waved = 0;
    int64_t total = 0;
    for (size_t j = c0; j < c1; ++j) {
      m.item[j - c0] = staged[j];
      m.shape[j - c0] = its[j].l.shape;
      tabd = std::max(tabd, bn::table_lds_bytes(its[j].a.net.R) / 8);
      waved = std::max(waved, bn::wave_lds_bytes(its[j].l.L, its[j].l.S, its[j].a.net.n) / 8);
      total += its[j].a.n_cells;
    }
    m.queue = queue + c0;
    m.tab_doubles = tabd;
    m.wave_doubles = waved;
    // workgroups of bw waves (the costliest network's choice, halved while
    // the LDS of a workgroup does not fit); as many per CU as LDS allows, up
    // to 4 W waves per CU
    int bw = its[c0].l.bw;
    while (bw > 1 && 8 * (tabd + (size_t)bw * waved) > lim.lds_block) bw /= 2;
    const size_t lds = 8 * (tabd + (size_t)bw * waved);
    if (lds > lim.lds_block)
      return fail(BN_EUNSUPPORTED, "network tables and working area exceed the LDS of a workgroup");
    m.block_waves = bw;
    int per_cu = std::max(1, 4 * W / bw);
    per_cu = std::min<int>(per_cu, (int)std::max<size_t>(1, lim.lds_cu / lds));
    int64_t grid = (int64_t)lim.cus * per_cu;
    // no more workgroups than there are cells to start
    const int64_t cells_per_wg = (int64_t)bw * 16;
    grid = std::max<int64_t>(1, std::min<int64_t>(grid, (total + cells_per_wg - 1) / cells_per_wg));
    // the items that factor in LDS keep J(y_J) per cell in their network's
    // areas when those hold this grid
    for (size_t j = c0; j < c1; ++j) {
      const int L = its[j].l.L, S = its[j].l.S, NP = L * S;
      bn::BurnArgs &ia = m.item[j - c0];
      ia.jws = nullptr;
      ia.jws_wave = 0;
      if ((S > 1 || NP >= 32) && its[j].net->jws) {
        const int64_t rows = NP >= 32 ? ia.net.n : NP;
        const int64_t per_wave = (int64_t)(64 / L) * rows * rows;
        if ((size_t)(grid * bw * per_wave) * 8 <= its[j].net->jws_bytes) {
          ia.jws = static_cast<double *>(its[j].net->jws);
          ia.jws_wave = per_wave;
        }
      }
    }
    launches.push_back([m, grid, W](hipStream_t s) { return bn::launch_multi(m, (int)grid, W, s); });
    c0 = c1;
  }
  // the generated networks' launches after the table-driven ones: a
  // generated workgroup takes a whole compute unit's LDS, so it fills the
  // units the long table-driven launches free towards their end
  for (auto &f : gen_launches) launches.push_back(std::move(f));
  SideStreams *side = nullptr;
  if (allow_fork && launches.size() > 1) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
      std::lock_guard<std::mutex> lk(g_side_mu);
      side = side_streams(dev);
    } else {
      (void)hipGetLastError();
    }
  }
  if (!side) {
    for (auto &f : launches)
      if ((e = f(st)) != hipSuccess)
        return fail(BN_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  } else {
    // fork: the side streams wait for what the caller's stream has enqueued
    // (counters, order and staging); join: the caller's stream waits for them
    std::lock_guard<std::mutex> lk(g_side_mu);
    if ((e = hipEventRecord(side->fork, st)) != hipSuccess)
      return fail(BN_EHIP, std::string("hipEventRecord failed: ") + hipGetErrorString(e));
    for (size_t j = 1; j < launches.size(); ++j)
      if ((e = hipStreamWaitEvent(side->s[j - 1], side->fork, 0)) != hipSuccess)
        return fail(BN_EHIP, std::string("hipStreamWaitEvent failed: ") + hipGetErrorString(e));
    for (size_t j = 0; j < launches.size(); ++j) {
      hipStream_t sj = j == 0 ? st : side->s[j - 1];
      if ((e = launches[j](sj)) != hipSuccess)
        return fail(BN_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    }
    for (size_t j = 1; j < launches.size(); ++j) {
      if ((e = hipEventRecord(side->done[j - 1], side->s[j - 1])) != hipSuccess ||
          (e = hipStreamWaitEvent(st, side->done[j - 1], 0)) != hipSuccess)
        return fail(BN_EHIP, std::string("stream join failed: ") + hipGetErrorString(e));
    }
  }
  if (o.order_cells) {
    for (size_t j = 0; j < its.size(); ++j) {
      e = bn::launch_stage_out(orig[j], staged[j], posv[j], st);
      if (e != hipSuccess)
        return fail(BN_EHIP, std::string("write-back launch failed: ") + hipGetErrorString(e));
    }
  }
  return BN_SUCCESS;
}

}  // namespace

extern "C" {

int burn_batch_multi(int32_t n_items, const bn_batch_item *items, double dt, double rtol,
                     double atol, const bn_burn_opts *opts, void *workspace,
                     size_t workspace_bytes, void *stream) {
  g_err.clear();
  return multi_impl(n_items, items, dt, rtol, atol, opts, workspace, workspace_bytes, stream,
                    true);
}

int burn_batch_multi_noalloc(int32_t n_items, const bn_batch_item *items, double dt,
                             double rtol, double atol, const bn_burn_opts *opts, void *stream) {
  g_err.clear();
  if (n_items < 0 || n_items > BN_MAX_ITEMS)
    return fail(BN_EINVAL, "n_items must be 0..BN_MAX_ITEMS");
  if (n_items > 0 && !items) return fail(BN_EINVAL, "null items");
  for (int j = 0; j < n_items; ++j)
    if (!items[j].net) return fail(BN_EINVAL, "null network in item " + std::to_string(j));
  const bool ordered = opts && opts->order_cells == 1;
  const size_t need = ordered ? burn_batch_multi_order_workspace_bytes(n_items, items)
                              : burn_batch_multi_workspace_bytes(n_items);
  if (need > (size_t)BN_NOALLOC_SCRATCH_BYTES)
    return fail(BN_EINVAL, "burn_batch_multi_noalloc: the launch needs " + std::to_string(need) +
                               " bytes of scratch, the library's static scratch holds " +
                               std::to_string((size_t)BN_NOALLOC_SCRATCH_BYTES) +
                               " (use burn_batch_multi with a workspace)");
  void *scratch = nullptr;
  const hipError_t e = bn::noalloc_scratch(&scratch);
  if (e != hipSuccess)
    return fail(BN_EHIP, std::string("hipGetSymbolAddress of the static scratch failed: ") +
                             hipGetErrorString(e));
  return multi_impl(n_items, items, dt, rtol, atol, opts, scratch,
                    (size_t)BN_NOALLOC_SCRATCH_BYTES, stream, false);
}

namespace {
int gen_desc_check(const bn_network_desc *d) {
  if (!d) return fail(BN_EINVAL, "null network description");
  const int N = d->n_species, R = d->n_reactions;
  if (N < 1 || R < 1 || !d->mass || !d->reactants || !d->products || !d->coef || !d->q)
    return fail(BN_EINVAL, "incomplete network description");
  if (R > BN_MAX_REACTIONS) return fail(BN_EUNSUPPORTED, "n_reactions exceeds BN_MAX_REACTIONS");
  for (int r = 0; r < 3 * R; ++r)
    if (d->reactants[r] < -1 || d->reactants[r] >= N || d->products[r] < -1 || d->products[r] >= N)
      return fail(BN_EINVAL, "species index out of range");
  if (!(d->c_v > 0.0) || !std::isfinite(d->c_v)) return fail(BN_EINVAL, "c_v must be positive");
  if (d->screen) return fail(BN_EUNSUPPORTED, "the generated body has no screening");
  return BN_SUCCESS;
}
}  // namespace

int bn_codegen_source(const bn_network_desc *desc, int32_t lanes_per_cell, char *buf, size_t cap,
                      size_t *len) {
  g_err.clear();
  if (int rc = gen_desc_check(desc)) return rc;
  const int lpc = gen_lanes(desc->n_species + 1, lanes_per_cell);
  if (!lpc) return fail(BN_EUNSUPPORTED, "no generated body for this system size and lanes_per_cell");
  bn::GenDesc g;
  fill_desc(desc, &g);
  const std::string src = bn::gen_source(g, lpc);
  if (len) *len = src.size() + 1;
  if (buf && cap) {
    const size_t m = std::min(cap - 1, src.size());
    std::memcpy(buf, src.data(), m);
    buf[m] = '\0';
  }
  return BN_SUCCESS;
}

int bn_codegen_prebuild(const bn_network_desc *desc, int32_t lanes_per_cell,
                        const char *cache_dir) {
  g_err.clear();
  if (int rc = gen_desc_check(desc)) return rc;
  if (!cache_dir || !*cache_dir) return fail(BN_EINVAL, "cache_dir is required");
  const int lpc = gen_lanes(desc->n_species + 1, lanes_per_cell);
  if (!lpc) return fail(BN_EUNSUPPORTED, "no generated body for this system size and lanes_per_cell");
  bn::GenDesc g;
  fill_desc(desc, &g);
  std::vector<char> code;
  std::string err;
  if (bn::gen_build(g, lpc, cache_dir, &code, &err) != 0) return fail(BN_EHIP, err);
  return BN_SUCCESS;
}

int bn_network_generate(bn_network *net, int32_t lanes_per_cell, const char *cache_dir) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (net->screened) return fail(BN_EUNSUPPORTED, "the generated body has no screening");
  const int lpc = gen_lanes(net->n, lanes_per_cell);
  if (!lpc) return fail(BN_EUNSUPPORTED, "no generated body for this system size and lanes_per_cell");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(BN_EHIP, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BN_EUNSUPPORTED, std::string("generated kernels are built for gfx950, not ") +
                                     prop.gcnArchName);
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  const size_t lds = bn::gen_lds_bytes(net->desc, lpc);
  if (lds > lim.lds_block)
    return fail(BN_EUNSUPPORTED, "the generated body's LDS exceeds a workgroup's");
  std::vector<char> code;
  std::string err;
  if (bn::gen_build(net->desc, lpc, cache_dir ? cache_dir : "", &code, &err) != 0)
    return fail(BN_EHIP, err);
  auto *g = new GenKernel();
  g->lpc = lpc;
  g->lds = lds;
  g->grid = lim.cus;
  g->n_lanes = (long long)lim.cus * 256;
  const int n = net->n;
  const size_t jb = (size_t)bn::gen_entries(net->desc, lpc) * g->n_lanes * sizeof(double);
  const size_t lb = (size_t)(n * n + 4 * n) * g->n_lanes * sizeof(double);
  if (hipModuleLoadData(&g->mod, code.data()) != hipSuccess) {
    free_gen(g);
    (void)hipGetLastError();
    return fail(BN_EHIP, "hipModuleLoadData of the generated kernel failed");
  }
  if (hipModuleGetFunction(&g->fn, g->mod, "bn_gen_burn") != hipSuccess) {
    free_gen(g);
    (void)hipGetLastError();
    return fail(BN_EHIP, "the generated code object has no bn_gen_burn");
  }
  if (hipMalloc(&g->jws, jb) != hipSuccess || hipMalloc(&g->lws, lb) != hipSuccess ||
      hipMalloc(&g->queue, 256) != hipSuccess) {
    free_gen(g);
    (void)hipGetLastError();
    return fail(BN_ENOMEM, "hipMalloc of the generated kernel's workspaces failed");
  }
  free_gen(net->gen);
  net->gen = g;
  net->body = BN_BODY_GENERATED;
  return BN_SUCCESS;
}

int bn_network_set_body(bn_network *net, int32_t body) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (body != BN_BODY_TABLE && body != BN_BODY_GENERATED)
    return fail(BN_EINVAL, "body must be BN_BODY_TABLE or BN_BODY_GENERATED");
  if (body == BN_BODY_GENERATED && !net->gen)
    return fail(BN_EINVAL, "the network has no generated kernel (bn_network_generate)");
  net->body = body;
  return BN_SUCCESS;
}

int bn_network_get_body(const bn_network *net, int32_t *body, int32_t *lanes_per_cell) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (body) *body = net->body;
  if (lanes_per_cell) *lanes_per_cell = net->gen ? net->gen->lpc : 0;
  return BN_SUCCESS;
}

int bn_network_set_persistent_launch(bn_network *net, int32_t lanes_per_cell,
                                     int32_t slots_per_lane, int32_t waves_per_simd,
                                     int32_t block_waves, double ms_per_cell) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (lanes_per_cell == 0) {
    net->pL = net->pS = net->pW = net->pbw = 0;
    return BN_SUCCESS;
  }
  if (waves_per_simd != 1 && waves_per_simd != 2)
    return fail(BN_EINVAL, "waves_per_simd must be 1 or 2");
  if ((waves_per_simd == 2 ? multi_shape_index(lanes_per_cell, slots_per_lane)
                           : multi1_shape_index(lanes_per_cell, slots_per_lane)) < 0)
    return fail(BN_EINVAL, "no persistent kernel with this shape at these waves per SIMD");
  if (lanes_per_cell * slots_per_lane < net->n)
    return fail(BN_EINVAL, "launch shape smaller than the system");
  if (block_waves < 1 || block_waves > 4) return fail(BN_EINVAL, "block_waves must be 1..4");
  net->pL = lanes_per_cell;
  net->pS = slots_per_lane;
  net->pW = waves_per_simd;
  net->pbw = block_waves;
  if (ms_per_cell > 0.0) net->ms_per_cell = ms_per_cell;
  return BN_SUCCESS;
}

int bn_network_get_persistent_launch(const bn_network *net, int32_t *lanes_per_cell,
                                     int32_t *slots_per_lane, int32_t *waves_per_simd,
                                     int32_t *block_waves) {
  g_err.clear();
  if (!net || !lanes_per_cell || !slots_per_lane || !waves_per_simd || !block_waves)
    return fail(BN_EINVAL, "null argument");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  const ItemLaunch l = item_launch(net, lim, 0);
  *lanes_per_cell = l.L;
  *slots_per_lane = l.S;
  *waves_per_simd = l.W;
  *block_waves = l.bw;
  return BN_SUCCESS;
}

int bn_network_set_launch(bn_network *net, int32_t lanes_per_cell, int32_t slots_per_lane,
                          int32_t block_waves) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (lanes_per_cell == 0) {
    net->L = net->S = net->block_waves = 0;
    net->ms_per_cell = 0.0;
    return BN_SUCCESS;
  }
  if (!plain_shape(lanes_per_cell, slots_per_lane))
    return fail(BN_EINVAL, "unknown launch shape");
  if (lanes_per_cell * slots_per_lane < net->n)
    return fail(BN_EINVAL, "launch shape smaller than the system");
  if (block_waves < 0 || block_waves > 4) return fail(BN_EINVAL, "block_waves must be 0..4");
  net->L = lanes_per_cell;
  net->S = slots_per_lane;
  net->block_waves = block_waves;
  return BN_SUCCESS;
}

int bn_network_get_launch(const bn_network *net, int32_t *lanes_per_cell,
                          int32_t *slots_per_lane, int32_t *block_waves) {
  g_err.clear();
  if (!net || !lanes_per_cell || !slots_per_lane || !block_waves)
    return fail(BN_EINVAL, "null argument");
  int L = net->L, S = net->S;
  if (!L) default_shape(net->n, &L, &S);
  *lanes_per_cell = L;
  *slots_per_lane = S;
  *block_waves = net->block_waves;
  return BN_SUCCESS;
}

int bn_network_autotune(bn_network *net, int64_t n_cells, const double *state,
                        const double *rho, const double *T, double dt, double rtol,
                        double atol, const double *log_mult, int32_t max_steps,
                        bn_tune_result *results, int32_t max_results, int32_t *n_results,
                        void *stream) {
  g_err.clear();
  if (n_results) *n_results = 0;
  if (!net) return fail(BN_EINVAL, "null network");
  if (n_cells < 1) return fail(BN_EINVAL, "autotune needs at least one cell");
  if (!state || !rho || !T) return fail(BN_EINVAL, "null state, rho or T");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  if (net->screened) return fail(BN_EUNSUPPORTED, "screened networks are not autotuned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t ybytes = (size_t)net->N * n_cells * 8, tbytes = (size_t)n_cells * 8;
  void *scratch = nullptr;
  if (hipMalloc(&scratch, ybytes + tbytes + (size_t)n_cells * 4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BN_ENOMEM, "hipMalloc of the autotune scratch failed");
  }
  double *Ys = static_cast<double *>(scratch);
  double *Ts = Ys + (size_t)net->N * n_cells;
  int32_t *sts = reinterpret_cast<int32_t *>(Ts + n_cells);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BN_SUCCESS;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = fail(BN_EHIP, "hipEventCreate failed");
  }
  double best = -1.0;
  int bL = 0, bS = 0, bbw = 0, nres = 0;
  const int n = net->n;
  for (int si = 0; rc == BN_SUCCESS && si < bn::N_PLAIN_SHAPES; ++si) {
    const int L = bn::PLAIN_SHAPES[si].L, S = bn::PLAIN_SHAPES[si].S;
    const int NP = L * S;
    if (NP < n || NP >= 4 * n + 16) continue;  // too small, or mostly padding
    for (int bw = 1; bw <= 4 && rc == BN_SUCCESS; bw *= 2) {
      if (lds_bytes(net->R, L, S, n, bw) > lim.lds_block) continue;
      bn::BurnArgs a{};
      a.net = net->tables;
      a.n_cells = n_cells;
      a.Y = Ys;
      a.rho = rho;
      a.T = Ts;
      a.log_mult = log_mult;
      a.status = sts;
      a.counters = nullptr;
      a.t_end = dt;
      a.rtol = rtol;
      a.atol = atol;
      a.max_steps = max_steps > 0 ? max_steps : 100000;
      double ms = 0.0;
      hipError_t e = hipSuccess;
      // the first run warms up; then the fastest of one timed run, or of
      // three when runs are short (a few milliseconds, where one run's
      // noise is comparable to the differences between shapes)
      int runs = 2;
      for (int rep = 0; rep < runs && e == hipSuccess; ++rep) {
        if ((e = hipMemcpyAsync(Ys, state, ybytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(Ts, T, tbytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) break;
        if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
        if ((e = bn::launch_plain(a, L, S, bw, st)) != hipSuccess) break;
        if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float f = 0.0f;
        if ((e = hipEventElapsedTime(&f, e0, e1)) != hipSuccess) break;
        if (rep == 1) {
          ms = f;
          if (f < 10.0f) runs = 4;
        } else if (rep > 1 && f < ms) {
          ms = f;
        }
      }
      if (results && nres < max_results) {
        results[nres].lanes_per_cell = L;
        results[nres].slots_per_lane = S;
        results[nres].block_waves = bw;
        results[nres].status = (int32_t)e;
        results[nres].ms = e == hipSuccess ? ms : -1.0;
      }
      ++nres;
      if (e != hipSuccess) {
        // a launch that does not fit is skipped; anything else is an error
        if (e == hipErrorInvalidValue || e == hipErrorInvalidConfiguration ||
            e == hipErrorLaunchOutOfResources) {
          (void)hipGetLastError();
          continue;
        }
        rc = fail(BN_EHIP, std::string("autotune launch failed: ") + hipGetErrorString(e));
        break;
      }
      if (best < 0.0 || ms < best) {
        best = ms;
        bL = L;
        bS = S;
        bbw = bw;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(scratch);
  if (n_results) *n_results = std::min(nres, max_results > 0 ? max_results : 0);
  if (rc != BN_SUCCESS) return rc;
  if (best < 0.0) return fail(BN_EUNSUPPORTED, "no launch shape fits this network");
  net->L = bL;
  net->S = bS;
  net->block_waves = bbw;
  net->ms_per_cell = best / (double)n_cells;
  return BN_SUCCESS;
}


int bn_network_autotune_persistent(bn_network *net, int64_t n_cells, const double *state,
                                   const double *rho, const double *T, double dt, double rtol,
                                   double atol, const double *log_mult, int32_t max_steps,
                                   bn_persistent_tune_result *results, int32_t max_results,
                                   int32_t *n_results, void *stream) {
  g_err.clear();
  if (n_results) *n_results = 0;
  if (!net) return fail(BN_EINVAL, "null network");
  if (n_cells < 1) return fail(BN_EINVAL, "autotune needs at least one cell");
  if (!state || !rho || !T) return fail(BN_EINVAL, "null state, rho or T");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  if (net->screened) return fail(BN_EUNSUPPORTED, "screened networks are not autotuned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t ybytes = (size_t)net->N * n_cells * 8, tbytes = (size_t)n_cells * 8;
  // the sample's working copies, then the ordered launch's workspace
  bn_batch_item item{};
  item.net = net;
  item.n_cells = n_cells;
  const size_t wsb = burn_batch_multi_order_workspace_bytes(1, &item);
  const size_t o_ws = align256(ybytes + tbytes + (size_t)n_cells * 4);
  void *scratch = nullptr;
  if (hipMalloc(&scratch, o_ws + wsb) != hipSuccess) {
    (void)hipGetLastError();
    return fail(BN_ENOMEM, "hipMalloc of the autotune scratch failed");
  }
  double *Ys = static_cast<double *>(scratch);
  double *Ts = Ys + (size_t)net->N * n_cells;
  int32_t *sts = reinterpret_cast<int32_t *>(Ts + n_cells);
  void *ws = static_cast<char *>(scratch) + o_ws;
  item.state = Ys;
  item.rho = rho;
  item.T = Ts;
  item.log_mult = log_mult;
  item.status = sts;
  item.counters = nullptr;
  bn_burn_opts o{};
  o.max_steps = max_steps > 0 ? max_steps : 100000;
  o.order_cells = 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = BN_SUCCESS;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = fail(BN_EHIP, "hipEventCreate failed");
  const int saved[4] = {net->pL, net->pS, net->pW, net->pbw};
  // the choices tuned are the table-driven persistent kernel's: a network
  // with its generated kernel selected is timed with the table body and
  // given its selection back at the end
  const int saved_body = net->body;
  net->body = BN_BODY_TABLE;
  // the choice derived without tuning (the network's plain shape, two waves
  // per SIMD when the LDS allows): a candidate replaces it only when it is
  // faster on the sample by more than the margin, since a sample's tail
  // weighs more than a full batch's and one timing per candidate is noisy
  ItemLaunch dflt{};
  {
    const int pw = net->pW;
    net->pW = 0;
    dflt = item_launch(net, lim, 0);
    net->pW = pw;
  }
  constexpr double kMargin = 0.97;
  double dflt_ms = -1.0;
  double best = -1.0;
  int best_c[4] = {0, 0, 0, 0};
  int nres = 0;
  const int n = net->n;
  for (int W = 2; W >= 1 && rc == BN_SUCCESS; --W) {
    for (int si = 0; si < bn::N_MULTI_SHAPES && rc == BN_SUCCESS; ++si) {
      const bn::ShapeLS sh = W == 2 ? bn::MULTI_SHAPES_2[si] : bn::MULTI_SHAPES_1[si];
      const int NP = sh.L * sh.S;
      if (NP < n || NP >= 4 * n + 16) continue;  // too small, or mostly padding
      for (int bw = 1; bw <= 4 && rc == BN_SUCCESS; bw *= 2) {
        if (lds_bytes(net->R, sh.L, sh.S, n, bw) > lim.lds_block) continue;
        net->pL = sh.L;
        net->pS = sh.S;
        net->pW = W;
        net->pbw = bw;
        double ms = 0.0;
        hipError_t e = hipSuccess;
        int brc = BN_SUCCESS;
        for (int rep = 0; rep < 2 && e == hipSuccess && brc == BN_SUCCESS; ++rep) {
          // the first run warms up
          if ((e = hipMemcpyAsync(Ys, state, ybytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) break;
          if ((e = hipMemcpyAsync(Ts, T, tbytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) break;
          if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
          brc = multi_impl(1, &item, dt, rtol, atol, &o, ws, wsb, stream, false);
          if (brc != BN_SUCCESS) break;
          if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
          if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
          float f = 0.0f;
          if ((e = hipEventElapsedTime(&f, e0, e1)) != hipSuccess) break;
          ms = f;
        }
        const bool okrun = e == hipSuccess && brc == BN_SUCCESS;
        if (results && nres < max_results) {
          bn_persistent_tune_result &r = results[nres];
          r.lanes_per_cell = sh.L;
          r.slots_per_lane = sh.S;
          r.waves_per_simd = W;
          r.block_waves = bw;
          r.status = okrun ? 0 : (brc != BN_SUCCESS ? brc : (int32_t)e);
          r.ms = okrun ? ms : -1.0;
        }
        ++nres;
        if (!okrun) {
          if (brc == BN_EUNSUPPORTED) continue;  // does not fit: skipped
          if (brc != BN_SUCCESS) {
            rc = brc;
            break;
          }
          rc = fail(BN_EHIP, std::string("autotune launch failed: ") + hipGetErrorString(e));
          break;
        }
        if (W == dflt.W && sh.L == dflt.L && sh.S == dflt.S && bw == dflt.bw) dflt_ms = ms;
        if (best < 0.0 || ms < best) {
          best = ms;
          best_c[0] = sh.L;
          best_c[1] = sh.S;
          best_c[2] = W;
          best_c[3] = bw;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  (void)hipFree(scratch);
  net->body = saved_body;
  if (best >= 0.0 && dflt_ms >= 0.0 && !(best < kMargin * dflt_ms)) {
    best = dflt_ms;
    best_c[0] = dflt.L;
    best_c[1] = dflt.S;
    best_c[2] = dflt.W;
    best_c[3] = dflt.bw;
  }
  if (n_results) *n_results = std::min(nres, max_results > 0 ? max_results : 0);
  if (rc != BN_SUCCESS || best < 0.0) {
    net->pL = saved[0];
    net->pS = saved[1];
    net->pW = saved[2];
    net->pbw = saved[3];
    if (rc != BN_SUCCESS) return rc;
    return fail(BN_EUNSUPPORTED, "no persistent launch fits this network");
  }
  net->pL = best_c[0];
  net->pS = best_c[1];
  net->pW = best_c[2];
  net->pbw = best_c[3];
  net->ms_per_cell = best / (double)n_cells;
  return BN_SUCCESS;
}


// ---- sensitivities -------------------------------------------------------

namespace {

struct AdjLayout {
  size_t stride;      // schedule doubles per cell
  int n_ckpt;
  size_t sched_bytes, ckpt_bytes, seg_bytes;
  size_t o_key, o_pos, o_order, o_hist;  // the cell order (costliest first)
  size_t o_soff;                         // per cell, its states' offset in the pool
  size_t o_queue;                        // the recording run's queue counter
  size_t total;                          // the minimum; a pool of states may follow
};

// schedules, checkpoints, the reverse sweep's segment states, then the cell
// order's sort keys, positions, order and bucket counters, the cells' state
// offsets (256-byte aligned); what the caller's workspace holds beyond this
// is the pool of corrected states
AdjLayout adj_layout(const bn_network *net, int64_t n_cells, int cap) {
  AdjLayout l{};
  l.stride = bn::adjoint_sched_stride(cap);
  l.n_ckpt = bn::adjoint_n_ckpt(cap);
  l.sched_bytes = 8 * l.stride * (size_t)n_cells;
  l.ckpt_bytes = 8 * (size_t)n_cells * l.n_ckpt * 7 * (size_t)net->n;
  l.seg_bytes = 8 * (size_t)n_cells * bn::adjoint_seg_doubles(net->n);
  size_t o = align256(l.sched_bytes + l.ckpt_bytes + l.seg_bytes);
  l.o_key = o;
  o += align256(4 * (size_t)n_cells);
  l.o_pos = o;
  o += align256(4 * (size_t)n_cells);
  l.o_order = o;
  o += align256(4 * (size_t)n_cells);
  l.o_hist = o;
  o += align256(8 * (size_t)bn::ORDER_BUCKETS);
  l.o_soff = o;
  o += align256(8 * (size_t)n_cells);
  l.o_queue = o;
  o += align256(8);
  l.total = o;
  return l;
}

int adj_check(const bn_network *net, int64_t n_cells, double dt, double rtol, double atol,
              int32_t max_steps, void *workspace, size_t workspace_bytes, int *dev_out) {
  if (!net) return fail(BN_EINVAL, "null network");
  if (n_cells < 0) return fail(BN_EINVAL, "n_cells < 0");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  if (max_steps < 1 || max_steps > 1000000)
    return fail(BN_EINVAL, "max_steps must be 1..1000000 for sensitivity runs");
  if (net->R > BN_ADJOINT_MAX_REACTIONS)
    return fail(BN_EUNSUPPORTED, "more reactions than BN_ADJOINT_MAX_REACTIONS");
  if (net->screened) return fail(BN_EUNSUPPORTED, "screened networks have no adjoint");
  if (n_cells == 0) return BN_SUCCESS;
  const AdjLayout l = adj_layout(net, n_cells, max_steps);
  if (!workspace || workspace_bytes < l.total)
    return fail(BN_EINVAL, "workspace missing or smaller than burn_batch_adjoint_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 8) return fail(BN_EINVAL, "workspace not 8-byte aligned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  if (bn::adjoint_lds_bytes(net->R, net->n, 1) > lim.lds_block)
    return fail(BN_EUNSUPPORTED, "network too large for the adjoint kernel's LDS");
  *dev_out = dev;
  return BN_SUCCESS;
}

bn::AdjArgs adj_args(const bn_network *net, int64_t n_cells, const double *state0,
                     const double *rho, const double *T0, double rtol, double atol,
                     const double *log_mult, int32_t max_steps, int32_t *status,
                     void *workspace, size_t workspace_bytes) {
  const AdjLayout l = adj_layout(net, n_cells, max_steps);
  bn::AdjArgs a{};
  a.net = net->tables;
  a.n_cells = n_cells;
  a.Y0 = state0;
  a.rho = rho;
  a.T0 = T0;
  a.log_mult = log_mult;
  a.status = status;
  a.sched = static_cast<double *>(workspace);
  a.sched_stride = (int64_t)l.stride;
  a.sched_cap = max_steps;
  a.ckpt = reinterpret_cast<double *>(static_cast<char *>(workspace) + l.sched_bytes);
  a.n_ckpt = l.n_ckpt;
  a.seg = reinterpret_cast<double *>(static_cast<char *>(workspace) + l.sched_bytes +
                                     l.ckpt_bytes);
  a.order = reinterpret_cast<const int32_t *>(static_cast<char *>(workspace) + l.o_order);
  a.soff = reinterpret_cast<int64_t *>(static_cast<char *>(workspace) + l.o_soff);
  a.states = reinterpret_cast<double *>(static_cast<char *>(workspace) + l.total);
  a.states_cap = workspace_bytes > l.total ? (int64_t)((workspace_bytes - l.total) / 8) : 0;
  a.rtol = rtol;
  a.atol = atol;
  return a;
}

// waves per workgroup of the adjoint kernels: as many (<= 4) as LDS allows
int adj_waves(const bn_network *net) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  DeviceLimits lim;
  if (device_limits(dev, &lim)) return 1;
  int w = 4;
  while (w > 1 && bn::adjoint_lds_bytes(net->R, net->n, w) > lim.lds_block) w /= 2;
  return w;
}

// register budget of the adjoint kernels: three waves per SIMD when the LDS
// lets twelve waves reside on a CU, else two
int adj_simd_waves(const bn_network *net, int waves) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  DeviceLimits lim;
  if (device_limits(dev, &lim)) return 2;
  const size_t per_block = bn::adjoint_lds_bytes(net->R, net->n, waves);
  const size_t resident = per_block ? (lim.lds_cu / per_block) * (size_t)waves : 0;
  return resident >= 12 ? 3 : 2;
}

}  // namespace

size_t burn_batch_adjoint_workspace_bytes(const bn_network *net, int64_t n_cells,
                                          int32_t max_steps) {
  if (!net || n_cells < 0 || max_steps < 1) return 0;
  return adj_layout(net, n_cells, max_steps).total;
}

size_t burn_batch_adjoint_states_bytes(const bn_network *net, int64_t total_steps) {
  if (!net || total_steps < 0) return 0;
  return 8 * (size_t)net->n * (size_t)total_steps;
}

int burn_batch_adjoint_forward(const bn_network *net, int64_t n_cells, const double *state0,
                               const double *rho, const double *T0, double dt, double rtol,
                               double atol, const double *log_mult, int32_t max_steps,
                               double *state_out, double *T_out, double *E_out,
                               int32_t *status, int32_t *counters, int32_t *replay_iters,
                               void *workspace, size_t workspace_bytes, void *stream) {
  g_err.clear();
  int dev = -1;
  if (int rc = adj_check(net, n_cells, dt, rtol, atol, max_steps, workspace, workspace_bytes,
                         &dev))
    return rc;
  if (n_cells == 0) return BN_SUCCESS;
  if (!state0 || !rho || !T0 || !state_out || !T_out || !E_out || !status)
    return fail(BN_EINVAL, "null array argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the recording run works on the output arrays
  if (hipMemcpyAsync(state_out, state0, 8 * (size_t)net->N * n_cells, hipMemcpyDeviceToDevice,
                     st) != hipSuccess ||
      hipMemcpyAsync(T_out, T0, 8 * (size_t)n_cells, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(BN_EHIP, "hipMemcpyAsync of the initial state failed");
  int L = net->L, S = net->S;
  if (!L || multi_shape_index(L, S) < 0) default_multi_shape(net->n, &L, &S);
  bn::BurnArgs b{};
  b.net = net->tables;
  b.n_cells = n_cells;
  b.Y = state_out;
  b.rho = rho;
  b.T = T_out;
  b.log_mult = log_mult;
  b.status = status;
  b.counters = counters;
  b.t_end = dt;
  b.rtol = rtol;
  b.atol = atol;
  b.max_steps = max_steps;
  bn::AdjArgs a = adj_args(net, n_cells, state0, rho, T0, rtol, atol, log_mult, max_steps, status,
                           workspace, workspace_bytes);
  b.sched = a.sched;
  b.sched_stride = a.sched_stride;
  b.sched_cap = a.sched_cap;
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  int bw = plain_waves(L, S) == 2 ? 1 : 2;
  while (bw > 1 && lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block) --bw;
  if (lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block)
    return fail(BN_EUNSUPPORTED, "network tables and working area exceed the LDS of a workgroup");
  // the recording run on a persistent grid with a cell queue (cells of
  // uneven length then share the lanes), the grid sized to the GPU as for
  // burn_batch_multi
  const size_t rlds = lds_bytes(net->R, L, S, net->n, bw);
  const int W = plain_waves(L, S);
  int per_cu = std::max(1, 4 * W / bw);
  per_cu = std::min<int>(per_cu, (int)std::max<size_t>(1, lim.lds_cu / rlds));
  const int64_t cells_per_wg = (int64_t)bw * (64 / L);
  const int64_t rgrid = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)lim.cus * per_cu, (n_cells + cells_per_wg - 1) / cells_per_wg));
  // shapes that factor in LDS keep J(y_J) per cell in the network's areas
  if ((S > 1 || L * S >= 32) && net->jws) {
    const int64_t rows = L * S >= 32 ? net->n : L * S;
    const int64_t per_wave = (int64_t)(64 / L) * rows * rows;
    if ((size_t)(rgrid * bw * per_wave) * 8 <= net->jws_bytes) {
      b.jws = static_cast<double *>(net->jws);
      b.jws_wave = per_wave;
    }
  }
  unsigned long long *rq = reinterpret_cast<unsigned long long *>(
      static_cast<char *>(workspace) + adj_layout(net, n_cells, max_steps).o_queue);
  hipError_t e = bn::launch_zero(rq, 1, st);
  if (e == hipSuccess) e = bn::launch_record_queue(b, L, S, bw, (int)rgrid, rq, st);
  if (e != hipSuccess) return fail(BN_EHIP, std::string("recording launch failed: ") + hipGetErrorString(e));
  {
    // replay and reverse sweep take the cells most recorded steps first
    const AdjLayout l = adj_layout(net, n_cells, max_steps);
    char *w = static_cast<char *>(workspace);
    e = bn::launch_adjoint_order(a, reinterpret_cast<float *>(w + l.o_key),
                                 reinterpret_cast<int32_t *>(w + l.o_pos),
                                 reinterpret_cast<unsigned *>(w + l.o_hist),
                                 reinterpret_cast<int32_t *>(w + l.o_order), st);
    if (e != hipSuccess)
      return fail(BN_EHIP, std::string("cell order launch failed: ") + hipGetErrorString(e));
    // the pool places of the corrected states the replay keeps
    e = bn::launch_adjoint_states(a, st);
    if (e != hipSuccess)
      return fail(BN_EHIP, std::string("state pool launch failed: ") + hipGetErrorString(e));
  }
  a.Yout = state_out;
  a.Tout = T_out;
  a.Eout = E_out;
  a.iters = replay_iters;
  const int aw = adj_waves(net);
  e = bn::launch_adjoint(a, false, aw, adj_simd_waves(net, aw), st);
  if (e != hipSuccess) return fail(BN_EHIP, std::string("replay launch failed: ") + hipGetErrorString(e));
  return BN_SUCCESS;
}

int burn_batch_adjoint_backward(const bn_network *net, int64_t n_cells, const double *state0,
                                const double *rho, const double *T0, double dt, double rtol,
                                double atol, const double *log_mult, int32_t max_steps,
                                const double *gY, const double *gE, double *grad,
                                const int32_t *status, void *workspace, size_t workspace_bytes,
                                void *stream) {
  g_err.clear();
  int dev = -1;
  if (int rc = adj_check(net, n_cells, dt, rtol, atol, max_steps, workspace, workspace_bytes,
                         &dev))
    return rc;
  if (n_cells == 0) return BN_SUCCESS;
  if (!state0 || !rho || !T0 || !gY || !gE || !grad || !status)
    return fail(BN_EINVAL, "null array argument");
  bn::AdjArgs a = adj_args(net, n_cells, state0, rho, T0, rtol, atol, log_mult, max_steps,
                           const_cast<int32_t *>(status), workspace, workspace_bytes);
  a.gY = gY;
  a.gE = gE;
  a.grad = grad;
  const int aw = adj_waves(net);
  const hipError_t e =
      bn::launch_adjoint(a, true, aw, adj_simd_waves(net, aw), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BN_EHIP, std::string("adjoint launch failed: ") + hipGetErrorString(e));
  return BN_SUCCESS;
}

int burn_batch_adjoint(const bn_network *net, int64_t n_cells, const double *state0,
                       const double *rho, const double *T0, double dt, double rtol, double atol,
                       const double *log_mult, int32_t max_steps, const double *gY,
                       const double *gE, double *state_out, double *T_out, double *E_out,
                       double *grad, int32_t *status, int32_t *counters,
                       int32_t *replay_iters, void *workspace, size_t workspace_bytes,
                       void *stream) {
  int rc = burn_batch_adjoint_forward(net, n_cells, state0, rho, T0, dt, rtol, atol, log_mult,
                                      max_steps, state_out, T_out, E_out, status, counters,
                                      replay_iters, workspace, workspace_bytes, stream);
  if (rc != BN_SUCCESS) return rc;
  return burn_batch_adjoint_backward(net, n_cells, state0, rho, T0, dt, rtol, atol, log_mult,
                                     max_steps, gY, gE, grad, status, workspace, workspace_bytes,
                                     stream);
}


int burn_batch_sdc(const bn_network *net, int64_t n_cells, double *state, const double *rho,
                   double *T, double dt, double rtol, double atol, const double *log_mult,
                   const double *source, int32_t *status, int32_t *counters,
                   const bn_burn_opts *opts, void *stream) {
  g_err.clear();
  if (!net) return fail(BN_EINVAL, "null network");
  if (n_cells < 0) return fail(BN_EINVAL, "n_cells < 0");
  if (int rc = check_tol(dt, rtol, atol)) return rc;
  bn_burn_opts o{};
  if (opts) o = *opts;
  if (o.max_steps <= 0) o.max_steps = 100000;
  if (o.block_waves < 0 || o.block_waves > 4) return fail(BN_EINVAL, "block_waves must be 0..4");
  int L = 0, S = 0;
  if (o.lanes_per_cell) {
    bool found = false;
    for (const bn::ShapeLS &sh : bn::MULTI_SHAPES_2)
      if (sh.L == o.lanes_per_cell && sh.L * sh.S >= net->n) {
        L = sh.L;
        S = sh.S;
        found = true;
        break;
      }
    if (!found) return fail(BN_EINVAL, "lanes_per_cell must be 0, 8, 16, 32 or 64 here");
  } else {
    L = net->L;
    S = net->S;
    if (!L || multi_shape_index(L, S) < 0) default_multi_shape(net->n, &L, &S);
  }
  if (n_cells == 0) return BN_SUCCESS;
  if (!state || !rho || !T || !source) return fail(BN_EINVAL, "null state, rho, T or source");
  if (net->screened) return fail(BN_EUNSUPPORTED, "screened networks are not supported here");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");
  DeviceLimits lim;
  if (int rc = device_limits(dev, &lim)) return rc;
  bn::BurnArgs a{};
  a.net = net->tables;
  a.n_cells = n_cells;
  a.Y = state;
  a.rho = rho;
  a.T = T;
  a.log_mult = log_mult;
  a.status = status;
  a.counters = counters;
  a.t_end = dt;
  a.rtol = rtol;
  a.atol = atol;
  a.max_steps = o.max_steps;
  a.src = source;
  int bw = o.block_waves ? o.block_waves : (plain_waves(L, S) == 2 ? 1 : 2);
  while (bw > 1 && lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block) --bw;
  if (lds_bytes(net->R, L, S, net->n, bw) > lim.lds_block)
    return fail(BN_EUNSUPPORTED, "network tables and working area exceed the LDS of a workgroup");
  const hipError_t e = bn::launch_source(a, L, S, bw, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BN_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BN_SUCCESS;
}

}  // extern "C"

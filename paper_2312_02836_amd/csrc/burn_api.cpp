// burn_api.cpp -- the C ABI declared in include/burn.h: network validation,
// device tables, argument checks and kernel dispatch.  No compute happens on
// the host: every step of the burn runs in the HIP kernels.

#include "burn.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "burn_internal.h"

namespace bn {
size_t plain_lds_bytes(const BurnArgs &a, int L, int S, int block_waves);
}

struct bn_network {
  int N = 0, R = 0, n = 0, nnz = 0;
  double c_v = 0.0;
  int device = 0;
  void *dev = nullptr;  // one allocation holding every table
  bn::NetTables tables{};
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
  for (int r = 0; r < R; ++r) {
    int c = 0;
    for (int i = 0; i < N; ++i) {
      const int v = nu_of(d, i, r);
      if (v) rout[8 * r + 1 + c++] = (i << 8) | (v & 0xff);
    }
    rout[8 * r] = c;
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
  // Layout of the device block: doubles first, then ints.
  const size_t nd = rtab.size() + q.size() + row_w.size();
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
  t.col_off = reinterpret_cast<const int *>(base + o_coloff);
  t.col_ent = reinterpret_cast<const int *>(base + o_colent);
  t.nu8 = reinterpret_cast<const signed char *>(base + o_nu8);
  t.rout = reinterpret_cast<const int *>(base + o_rout);
  *out = net;
  return BN_SUCCESS;
}

void bn_network_destroy(bn_network *net) {
  if (!net) return;
  if (net->dev) (void)hipFree(net->dev);
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
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(BN_EINVAL, "dt must be positive and finite");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(BN_EINVAL, "rtol must be positive");
  if (!(atol >= 0.0) || !std::isfinite(atol)) return fail(BN_EINVAL, "atol must be >= 0");
  if (n_cells == 0) return BN_SUCCESS;
  if (!state || !rho || !T) return fail(BN_EINVAL, "null state, rho or T");
  bn_burn_opts o{};
  if (opts) o = *opts;
  if (o.max_steps <= 0) o.max_steps = 100000;
  if (o.lanes_per_cell != 0 && o.lanes_per_cell != 4 && o.lanes_per_cell != 8 &&
      o.lanes_per_cell != 16 && o.lanes_per_cell != 64)
    return fail(BN_EINVAL, "lanes_per_cell must be 0, 4, 8, 16 or 64");
  if (o.block_waves < 0 || o.block_waves > 4) return fail(BN_EINVAL, "block_waves must be 0..4");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(BN_EHIP, "hipGetDevice failed");
  if (dev != net->device) return fail(BN_EINVAL, "network was created on another device");

  int L = 0, S = 0;
  if (!bn::choose_shape(net->n, o.lanes_per_cell, &L, &S))
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

  int bw = o.block_waves;
  if (bw == 0) {
    bw = 2;
    while (bw > 1 && bn::plain_lds_bytes(a, L, S, bw) > 64 * 1024) --bw;
  }
  if (bn::plain_lds_bytes(a, L, S, bw) > 64 * 1024)
    return fail(BN_EUNSUPPORTED, "network tables too large for LDS");
  const hipError_t e = bn::launch_plain(a, L, S, bw, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(BN_EHIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return BN_SUCCESS;
}

int burn_batch(const bn_network *net, int64_t n_cells, double *state, const double *rho,
               double *T, double dt, double rtol, double atol, const double *log_mult,
               int32_t *status, int32_t *counters, void *stream) {
  return burn_batch_ex(net, n_cells, state, rho, T, dt, rtol, atol, log_mult, status, counters,
                       nullptr, stream);
}

}  // extern "C"

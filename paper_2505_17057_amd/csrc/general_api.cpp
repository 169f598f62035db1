// The general-scheme solver behind mfd_general_*: the MMFD scheme of
// Eq. (2-2-1) with any stencil reach m and number of time levels n for the
// linear CDE, on any lattice of Appendix A (rD3Q27 included), square or
// rectangular, and for Burgers' equation and the NSE on the square lattices
// of up to 19 velocities; periodic.  A ring of n + 1 device levels; one
// kernel launch per step (kernels_general.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/mfd.h"
#include "general.h"
#include "mfd_internal.h"
#include "scheme.h"

struct mfd_general {
  mfd_grid grid{};
  mfd::Grid G{};
  mfd::Consts consts{};
  int eq = MFD_LCDE, nf = 1;
  int m = 1, nl = 1;
  double a[mfd::kGenMaxLevels][2 * mfd::kGenMaxM + 1] = {};
  double ab[mfd::kGenMaxLevels][2 * mfd::kGenMaxM + 1] = {};
  void *lev[mfd::kGenMaxLevels + 1] = {nullptr};
  int ring[mfd::kGenMaxLevels + 1] = {0};  // slot of level l (l = nl: the spare)
  void *d_gc = nullptr;
  hipStream_t stream = nullptr;
  bool state_set = false, sticky = false;
  std::string err;

  int fail(int code, const char *fmt, ...) {
    char b[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(b, sizeof(b), fmt, ap);
    va_end(ap);
    err = b;
    return code;
  }
  int hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return MFD_OK;
    sticky = true;
    return fail(MFD_E_HIP, "%s: %s", what, hipGetErrorString(e));
  }
  int64_t elem() const { return grid.precision == MFD_FP64 ? 8 : 4; }
  void *slot(int level) const { return lev[ring[level]]; }
};

namespace mfd {
namespace {

template <typename T>
GenC<T> gen_constants(const mfd_general &g) {
  GenC<T> c;
  std::memset(&c, 0, sizeof(c));
  c.m = g.m;
  c.nl = g.nl;
  const int m = g.m;
  for (int l = 0; l < g.nl; ++l) {
    double s = 0.0;
    for (int kk = 0; kk < 2 * m + 1; ++kk) s = s + g.a[l][kk];
    c.A[l] = (T)s;
    for (int k = 1; k <= m; ++k) {
      const double ap = g.a[l][m + k] + g.a[l][m - k];
      const double am = g.a[l][m + k] - g.a[l][m - k];
      for (int p = 0; p < g.consts.npair; ++p) {
        c.Cp[l][k - 1][p] = (T)(ap * g.consts.ubp[p]);
        c.Cm[l][k - 1][p] = (T)(am * g.consts.ubm[p]);
      }
    }
  }
  return c;
}

template <typename T>
GenNL<T> gen_nl_constants(const mfd_general &g) {
  GenNL<T> c;
  std::memset(&c, 0, sizeof(c));
  c.m = g.m;
  c.nl = g.nl;
  const int m = g.m;
  for (int l = 0; l < g.nl; ++l) {
    double s = 0.0, sb = 0.0;
    for (int kk = 0; kk < 2 * m + 1; ++kk) {
      s = s + g.a[l][kk];
      sb = sb + g.ab[l][kk];
    }
    c.A[l] = (T)s;
    c.Ab[l] = (T)sb;
    for (int k = 1; k <= m; ++k) {
      c.ap[l][k - 1] = (T)(g.a[l][m + k] + g.a[l][m - k]);
      c.am[l][k - 1] = (T)(g.a[l][m + k] - g.a[l][m - k]);
      c.abp[l][k - 1] = (T)(g.ab[l][m + k] + g.ab[l][m - k]);
      c.abm[l][k - 1] = (T)(g.ab[l][m + k] - g.ab[l][m - k]);
    }
  }
  return c;
}

template <typename T>
int general_steps(mfd_general *g, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; ++s) {
    GenLevels<T> lv{};
    for (int l = 0; l < g->nl; ++l) lv.p[l] = (const T *)g->slot(l);
    hipError_t e =
        g->eq == MFD_LCDE
            ? launch_general_step<T>(g->consts.lattice, g->m, lv, (T *)g->slot(g->nl), g->G.n,
                                     (const GenC<T> *)g->d_gc, g->stream)
            : launch_general_nl_step<T>(g->consts, g->m, lv, (T *)g->slot(g->nl), g->G.n,
                                        (const GenNL<T> *)g->d_gc, g->stream);
    if (e != hipSuccess) return g->hip(e, "general step launch");
    // the new level becomes level 0; the oldest one's slot the spare
    const int spare = g->ring[g->nl];
    for (int l = g->nl; l > 0; --l) g->ring[l] = g->ring[l - 1];
    g->ring[0] = spare;
  }
  return MFD_OK;
}

}  // namespace
}  // namespace mfd

using namespace mfd;

#define GENERAL_OR_ARG(g) \
  do {                    \
    if (!(g)) return MFD_E_ARG; \
  } while (0)

extern "C" int mfd_general_create(mfd_general **out, const mfd_grid *grid, int lattice,
                                  const double d0[3], const double spacing[3], int eq_code,
                                  const mfd_eq_params *eq, int32_t m, int32_t n, const double *a,
                                  const double *ab, double dt) {
  if (!out) return MFD_E_ARG;
  *out = nullptr;
  if (!grid || !eq || !a) return MFD_E_ARG;
  if (eq_code != MFD_LCDE && eq_code != MFD_BURGERS && eq_code != MFD_NSE) return MFD_E_UNSUPPORTED;
  // the nonlinear equations: square lattices of at most 19 velocities
  if (eq_code != MFD_LCDE && (spacing || lattice == MFD_D3Q27)) return MFD_E_UNSUPPORTED;
  if (eq_code == MFD_NSE && grid->dim < 2) return MFD_E_UNSUPPORTED;
  if (grid->dim < 1 || grid->dim > 3 || grid->form != MFD_MMFD || grid->boundary != MFD_PERIODIC ||
      (grid->precision != MFD_FP64 && grid->precision != MFD_FP32))
    return MFD_E_UNSUPPORTED;
  if (m < 1 || m > kGenMaxM || n < 1 || n > kGenMaxLevels || !(dt > 0.0)) return MFD_E_ARG;
  for (int x = 0; x < 3; ++x)
    if (grid->n[x] < 1 || (x >= grid->dim && grid->n[x] != 1)) return MFD_E_ARG;
  if (grid->n[1] > 4 * 65535 || grid->n[2] > 65535) return MFD_E_ARG;  // launch-grid limits
  for (int i = 0; i < n * (2 * m + 1); ++i)
    if (!std::isfinite(a[i]) || (ab && !std::isfinite(ab[i]))) return MFD_E_ARG;
  // the scheme's moments (Eq. (4-2-00a), the new level at q = 0)
  double A00 = 0.0, A10 = 0.0, A11 = 0.0, A22 = 0.0;
  for (int l = 0; l < n; ++l)
    for (int kk = 0; kk < 2 * m + 1; ++kk) {
      const int k = kk - m;
      const double v = a[l * (2 * m + 1) + kk];
      A00 = A00 + v;
      A10 = A10 + (double)(-(l + 1)) * v;
      A11 = A11 + (double)k * v;
      A22 = A22 + 0.5 * (double)(k * k) * v;
    }
  // the linear CDE maps K through -A10 / A22
  if (eq_code == MFD_LCDE && (!(A10 < 0.0) || !(A22 > 0.0))) return MFD_E_ARG;
  SchemeInput in;
  std::memset(&in, 0, sizeof(in));
  in.lattice = lattice;
  in.d0 = d0 && d0[0] > 0.0 ? d0[0] : 1.0 / 3.0;
  in.eq = eq_code == MFD_LCDE ? kLCDE : (eq_code == MFD_BURGERS ? kBurgers : kNSE);
  in.kind = MFD_TWO_LEVEL;
  in.a[0] = 1.0;  // the per-pair tables take the general scheme's own ratio
  in.ab[0] = 1.0;
  in.rho0 = eq->rho0;
  in.he_luo = eq->he_luo;
  in.dt = dt;
  in.dx = grid->dx;
  for (int x = 0; x < 3; ++x) in.u[x] = eq->u[x];
  for (int i = 0; i < 9; ++i) in.K[i] = eq->K[i];
  in.lambda_bar = eq->lambda_bar;
  in.beta = eq_code == MFD_BURGERS && eq->beta != 0.0 ? eq->beta : 1.0;
  in.ratio = eq_code == MFD_LCDE ? -A10 / A22 : 0.0;
  if (spacing) {
    in.rect = 1;
    for (int x = 0; x < 3; ++x) {
      const int s = x < grid->dim ? x : 0;
      in.d0v[x] = d0 ? d0[s] : 1.0 / 3.0;
      in.dxv[x] = spacing[s];
      if (!(in.d0v[x] > 0.0 && in.d0v[x] < 1.0) || !(in.dxv[x] > 0.0)) return MFD_E_ARG;
    }
  } else if (!(grid->dx > 0.0) || !(in.d0 < 1.0)) {
    return MFD_E_ARG;
  }
  mfd_general *g = new mfd_general();
  g->grid = *grid;
  int rc = build_consts(in, g->consts);
  if (rc == MFD_OK && g->consts.dim != grid->dim) rc = MFD_E_ARG;
  if (rc != MFD_OK) {
    delete g;
    return rc;
  }
  g->eq = eq_code;
  g->nf = eq_code == MFD_NSE ? 1 + grid->dim : 1;
  g->m = m;
  g->nl = n;
  for (int l = 0; l < n; ++l)
    for (int kk = 0; kk < 2 * m + 1; ++kk) {
      g->a[l][kk] = a[l * (2 * m + 1) + kk];
      g->ab[l][kk] = ab ? ab[l * (2 * m + 1) + kk] : g->a[l][kk];
    }
  g->G.N = 1;
  for (int x = 0; x < 3; ++x) {
    g->G.n[x] = grid->n[x];
    g->G.N *= grid->n[x];
  }
  const size_t bytes = (size_t)(g->nf * g->G.N * g->elem());
  for (int l = 0; l <= n; ++l) {
    g->ring[l] = l;
    if (dev_malloc(&g->lev[l], bytes) != hipSuccess) {
      (void)hipGetLastError();
      for (int i = 0; i < l; ++i) dev_free(g->lev[i]);
      delete g;
      return MFD_E_OOM;
    }
  }
  hipError_t e;
  auto upload = [&](const void *c, size_t sz) {
    hipError_t r = dev_malloc(&g->d_gc, sz);
    if (r == hipSuccess) r = hipMemcpy(g->d_gc, c, sz, hipMemcpyHostToDevice);
    return r;
  };
  if (eq_code == MFD_LCDE) {
    if (grid->precision == MFD_FP64) {
      const GenC<double> c = gen_constants<double>(*g);
      e = upload(&c, sizeof(c));
    } else {
      const GenC<float> c = gen_constants<float>(*g);
      e = upload(&c, sizeof(c));
    }
  } else if (grid->precision == MFD_FP64) {
    const GenNL<double> c = gen_nl_constants<double>(*g);
    e = upload(&c, sizeof(c));
  } else {
    const GenNL<float> c = gen_nl_constants<float>(*g);
    e = upload(&c, sizeof(c));
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    for (int l = 0; l <= n; ++l) dev_free(g->lev[l]);
    dev_free(g->d_gc);
    delete g;
    return MFD_E_OOM;
  }
  *out = g;
  // consistency warnings (Eq. (4-2-00a): A00 = 1; the advection needs A11 = A10)
  if (std::fabs(A00 - 1.0) > 1e-12 || (eq_code == MFD_LCDE && std::fabs(A11 - A10) > 1e-12))
    return MFD_W_INCONSISTENT;
  return MFD_OK;
}

extern "C" int mfd_general_destroy(mfd_general *g) {
  if (!g) return MFD_OK;
  (void)hipStreamSynchronize(g->stream);
  for (int l = 0; l <= g->nl; ++l) dev_free(g->lev[l]);
  dev_free(g->d_gc);
  delete g;
  return MFD_OK;
}

extern "C" const char *mfd_general_last_error(const mfd_general *g) {
  return g ? g->err.c_str() : "null general solver";
}

extern "C" int mfd_general_set_stream(mfd_general *g, void *stream) {
  GENERAL_OR_ARG(g);
  g->stream = (hipStream_t)stream;
  return MFD_OK;
}

extern "C" int mfd_general_set_level(mfd_general *g, int32_t level, const void *src, int64_t bytes,
                                     int on_device) {
  GENERAL_OR_ARG(g);
  if (g->sticky) return g->fail(MFD_E_HIP, "general solver is in a failed HIP state");
  if (!src) return g->fail(MFD_E_ARG, "null source");
  if (level < 0 || level >= g->nl) return g->fail(MFD_E_ARG, "level must lie in [0, %d)", g->nl);
  if (level > 0 && !g->state_set) return g->fail(MFD_E_ORDER, "set level 0 first");
  if (bytes != g->nf * g->G.N * g->elem())
    return g->fail(MFD_E_ARG, "expected %lld bytes, got %lld",
                   (long long)(g->nf * g->G.N * g->elem()), (long long)bytes);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  // level 0 also fills the older levels (phi^(-l) = phi^0 until set)
  const int last = level == 0 ? g->nl - 1 : level;
  for (int l = level; l <= last; ++l) {
    hipError_t e = hipMemcpyAsync(g->slot(l), src, (size_t)bytes, kind, g->stream);
    if (e != hipSuccess) return g->hip(e, "hipMemcpyAsync (in)");
  }
  hipError_t e = hipStreamSynchronize(g->stream);
  if (e != hipSuccess) return g->hip(e, "hipStreamSynchronize");
  g->state_set = true;
  return MFD_OK;
}

extern "C" int mfd_general_get_level(mfd_general *g, int32_t level, void *dst, int64_t bytes,
                                     int on_device) {
  GENERAL_OR_ARG(g);
  if (g->sticky) return g->fail(MFD_E_HIP, "general solver is in a failed HIP state");
  if (!g->state_set) return g->fail(MFD_E_ORDER, "state not set");
  if (!dst) return g->fail(MFD_E_ARG, "null destination");
  if (level < 0 || level >= g->nl) return g->fail(MFD_E_ARG, "level must lie in [0, %d)", g->nl);
  if (bytes != g->nf * g->G.N * g->elem())
    return g->fail(MFD_E_ARG, "expected %lld bytes, got %lld",
                   (long long)(g->nf * g->G.N * g->elem()), (long long)bytes);
  hipError_t e = hipMemcpyAsync(dst, g->slot(level), (size_t)bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return g->hip(e, "level copy");
}

extern "C" int mfd_general_step(mfd_general *g, int64_t nsteps) {
  GENERAL_OR_ARG(g);
  if (g->sticky) return g->fail(MFD_E_HIP, "general solver is in a failed HIP state");
  if (nsteps < 0) return g->fail(MFD_E_ARG, "nsteps < 0");
  if (!g->state_set) return g->fail(MFD_E_ORDER, "state not set");
  return g->grid.precision == MFD_FP64 ? general_steps<double>(g, nsteps)
                                       : general_steps<float>(g, nsteps);
}

extern "C" int mfd_general_synchronize(mfd_general *g) {
  GENERAL_OR_ARG(g);
  return g->hip(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
}

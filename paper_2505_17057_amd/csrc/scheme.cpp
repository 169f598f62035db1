// Host-side algebra of the MesoFD / MMFD schemes: lattice tables
// (Appendix A), coefficient moments (Eq. (4-2-00)), the closed-form
// constraint solve (Eq. (X)), presets, the PDE-coefficient mapping
// (alpha = -(A22/A10) dt beta c_s^2, nu = -(Abar22/Abar10) dt c_s^2), the
// derived per-step constants and the linear stability analysis
// (Eq. (TforMMFD-3), Theorems 1-3).
//
// Every constant is formed in binary64 in a fixed expression order (left to
// right as written); the FP64 kernels consume them unchanged.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "../../include/mfd.h"
#include "mfd_internal.h"
#include "scheme.h"

namespace mfd {

namespace {

template <class L>
void copy_lattice(Consts &c) {
  c.dim = L::D;
  c.q = L::Q;
  c.npair = L::P;
  for (int j = 0; j < L::Q; ++j)
    for (int a = 0; a < 3; ++a) c.e[j][a] = L::E[j][a];
  for (int p = 0; p < L::P; ++p) c.pair[p] = L::PR[p];
}

constexpr int kOffA[3] = {0, 0, 1};
constexpr int kOffB[3] = {1, 2, 2};

// e_j . B, e in {-1, 0, 1}: signed accumulation from zero.
double edot(const Consts &c, int j, const double *B) {
  double s = 0.0;
  for (int a = 0; a < c.dim; ++a) {
    if (c.e[j][a] == 1) s = s + B[a];
    else if (c.e[j][a] == -1) s = s - B[a];
  }
  return s;
}

// Q~_j : C with the diagonal terms first (axis order), then the distinct
// off-diagonal pairs (0,1), (0,2), (1,2) with e_a e_b != 0.
double quad(const Consts &c, int j, const double *C) {
  double t = c.qd[j][0] * C[0];
  for (int a = 1; a < c.dim; ++a) t = t + c.qd[j][a] * C[a * 3 + a];
  const int no = c.dim == 1 ? 0 : (c.dim == 2 ? 1 : 3);
  for (int o = 0; o < no; ++o)
    if (c.qo[j][o] != 0.0) t = t + c.qo[j][o] * C[kOffA[o] * 3 + kOffB[o]];
  return t;
}

}  // namespace

int lattice_weights_v(int lattice, const double d0v[3], Consts &c) {
  const double d0 = d0v[0], dx = d0v[0], dy = d0v[1], dz = d0v[2];
  switch (lattice) {
    case MFD_D1Q3:
      copy_lattice<LatD1Q3>(c);
      c.w[0] = 1.0 - dx;
      c.w[1] = dx / 2.0;
      c.w[2] = dx / 2.0;
      break;
    case MFD_D2Q5:
      copy_lattice<LatD2Q5>(c);
      c.w[0] = 1.0 - dx - dy;
      c.w[1] = dx / 2.0;
      c.w[3] = c.w[1];
      c.w[2] = dy / 2.0;
      c.w[4] = c.w[2];
      break;
    case MFD_D2Q9:
      copy_lattice<LatD2Q9>(c);
      c.w[0] = (1.0 - dx) * (1.0 - dy);
      c.w[1] = dx * (1.0 - dy) / 2.0;
      c.w[3] = c.w[1];
      c.w[2] = (1.0 - dx) * dy / 2.0;
      c.w[4] = c.w[2];
      c.w[5] = dx * dy / 4.0;
      c.w[6] = c.w[7] = c.w[8] = c.w[5];
      break;
    case MFD_D3Q19: {
      copy_lattice<LatD3Q19>(c);
      c.w[0] = 1.0 - dx - dy - dz + dx * dy + dx * dz + dy * dz;
      c.w[1] = c.w[4] = dx * (1.0 - dy - dz) / 2.0;
      c.w[2] = c.w[5] = dy * (1.0 - dx - dz) / 2.0;
      c.w[3] = c.w[6] = dz * (1.0 - dx - dy) / 2.0;
      for (int j = 7; j <= 10; ++j) c.w[j] = dx * dy / 4.0;
      for (int j = 11; j <= 14; ++j) c.w[j] = dx * dz / 4.0;
      for (int j = 15; j <= 18; ++j) c.w[j] = dy * dz / 4.0;
      break;
    }
    case MFD_D2Q5II:
      if (dy != d0) return MFD_E_UNSUPPORTED;
      copy_lattice<LatD2Q5II>(c);
      c.w[0] = 1.0 - d0;
      for (int j = 1; j <= 4; ++j) c.w[j] = d0 / 4.0;
      break;
    case MFD_D3Q7:
      copy_lattice<LatD3Q7>(c);
      c.w[0] = 1.0 - dx - dy - dz;
      c.w[1] = c.w[4] = dx / 2.0;
      c.w[2] = c.w[5] = dy / 2.0;
      c.w[3] = c.w[6] = dz / 2.0;
      break;
    case MFD_D3Q27:
      copy_lattice<LatD3Q27>(c);
      c.w[0] = (1.0 - dx) * (1.0 - dy) * (1.0 - dz);
      c.w[1] = c.w[4] = dx * (1.0 - dy) * (1.0 - dz) / 2.0;
      c.w[2] = c.w[5] = dy * (1.0 - dx) * (1.0 - dz) / 2.0;
      c.w[3] = c.w[6] = dz * (1.0 - dx) * (1.0 - dy) / 2.0;
      for (int j = 7; j <= 10; ++j) c.w[j] = dx * dy * (1.0 - dz) / 4.0;
      for (int j = 11; j <= 14; ++j) c.w[j] = dx * dz * (1.0 - dy) / 4.0;
      for (int j = 15; j <= 18; ++j) c.w[j] = dy * dz * (1.0 - dx) / 4.0;
      for (int j = 19; j <= 26; ++j) c.w[j] = dx * dy * dz / 8.0;
      break;
    case MFD_D3Q9:
      if (dy != d0 || dz != d0) return MFD_E_UNSUPPORTED;
      copy_lattice<LatD3Q9>(c);
      c.w[0] = 1.0 - d0;
      for (int j = 1; j <= 8; ++j) c.w[j] = d0 / 8.0;
      break;
    default:
      return MFD_E_ARG;
  }
  c.lattice = lattice;
  c.d0 = d0;
  for (int j = 0; j < c.q; ++j)
    if (!(c.w[j] > 0.0)) return MFD_E_ARG;
  return MFD_OK;
}

int lattice_weights(int lattice, double d0, Consts &c) {
  const double dv[3] = {d0, d0, d0};
  return lattice_weights_v(lattice, dv, c);
}

int build_consts(const SchemeInput &in, Consts &c) {
  std::memset(&c, 0, sizeof(c));
  // d0 and spacing per axis (rectangular lattice: the linear CDE only)
  double d0v[3] = {in.d0, in.d0, in.d0}, dxv[3] = {in.dx, in.dx, in.dx};
  if (in.rect) {
    if (in.eq != kLCDE) return MFD_E_UNSUPPORTED;
    for (int x = 0; x < 3; ++x) {
      d0v[x] = in.d0v[x];
      dxv[x] = in.dxv[x];
    }
  }
  int rc = lattice_weights_v(in.lattice, d0v, c);
  if (rc) return rc;
  const double d0 = in.d0;
  c.eq = in.eq;
  c.inv_d0 = 1.0 / d0;
  // Eq. (3-4) in lattice units, per axis
  for (int j = 0; j < c.q; ++j) {
    for (int a = 0; a < 3; ++a) {
      const double ea = (double)c.e[j][a];
      c.qd[j][a] = (ea * ea - d0v[a]) / (d0v[a] * (1.0 - d0v[a]));
    }
    for (int o = 0; o < 3; ++o)
      c.qo[j][o] =
          (double)(c.e[j][kOffA[o]] * c.e[j][kOffB[o]]) / (d0v[kOffA[o]] * d0v[kOffB[o]]);
    c.w1[j] = c.w[j] * c.inv_d0;
  }
  const double *a = in.a, *ah = in.ah, *ab = in.ab, *abh = in.abh;
  c.A0 = a[0] + a[1] + a[2];
  c.Ah0 = ah[0] + ah[1] + ah[2];
  c.Ab0 = ab[0] + ab[1] + ab[2];
  c.Abh0 = abh[0] + abh[1] + abh[2];
  c.ap = a[2] + a[0];
  c.am = a[2] - a[0];
  c.ahp = ah[2] + ah[0];
  c.ahm = ah[2] - ah[0];
  c.abp = ab[2] + ab[0];
  c.abm = ab[2] - ab[0];
  c.abhp = abh[2] + abh[0];
  c.abhm = abh[2] - abh[0];
  if (in.multiset) {
    c.ap = in.ae[2] + in.ae[0];
    c.am = in.ao[2] - in.ao[0];
    c.ahp = in.aeh[2] + in.aeh[0];
    c.ahm = in.aoh[2] - in.aoh[0];
    c.multiset = 1;
  }
  for (int k = 0; k < 3; ++k) {
    c.a[k] = a[k];
    c.ah[k] = in.kind == MFD_THREE_LEVEL ? ah[k] : 0.0;
  }
  c.three = in.kind == MFD_THREE_LEVEL;
  c.three_stencil = c.three && (c.ahp != 0.0 || c.ahm != 0.0 || c.abhp != 0.0 || c.abhm != 0.0);

  if (in.eq == kWaveInput) {
    // wave equation (Example 3 of the paper): the linear EDF
    // f_j = w_j phi [1 + (beta - 1)(|e_j|^2 - dim d0) / (2 d0)], no velocity;
    // it runs the linear CDE kernels with this constant table
    c.eq = kLCDE;
    c.wave = 1;
    for (int j = 0; j < c.q; ++j) {
      double e2 = 0.0;
      for (int x = 0; x < 3; ++x) e2 = e2 + (double)(c.e[j][x] * c.e[j][x]);
      const double t = (e2 - (double)c.dim * d0) / (2.0 * d0);
      c.ubar[j] = c.w[j] * (1.0 + (in.beta - 1.0) * t);
    }
    for (int p = 0; p < c.npair; ++p) {
      const int j = c.pair[p];
      c.ubp[p] = c.ubar[j];
      c.ubm[p] = 0.0;
      c.Cp[p] = c.ap * c.ubp[p];
      c.Cm[p] = 0.0;
      c.Chp[p] = c.ahp * c.ubp[p];
      c.Chm[p] = 0.0;
    }
    c.theta = 1.0;
    c.th1 = 0.0;
    c.den = 1.0;
    c.inv_den = 1.0;
  } else if (in.eq == kLCDE) {
    const double A10 = -c.Ah0 - 1.0;
    const double A22 = 0.5 * (c.ap + c.ahp);
    const double ratio = in.ratio > 0.0 ? in.ratio : -A10 / A22;
    // lattice units per axis: u_a dt / dx_a, K_ab dt / (dx_a dx_b)
    for (int x = 0; x < 3; ++x) c.uh[x] = in.u[x] * in.dt / dxv[x];
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) c.kh[x * 3 + y] = in.K[x * 3 + y] * in.dt / (dxv[x] * dxv[y]);
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) {
        double v = ratio * c.kh[x * 3 + y];
        if (x == y) v = v - d0v[x];
        if (in.lambda_bar) v = v + c.uh[x] * c.uh[y];
        c.Ch[x * 3 + y] = v;
      }
    // c~_j . uh: the square lattice divides the sum by d0 once, the
    // rectangular one each axis by its own d0
    double ut[3];
    for (int x = 0; x < 3; ++x) ut[x] = c.uh[x] / d0v[x];
    for (int j = 0; j < c.q; ++j) {
      const double lin = in.rect ? edot(c, j, ut) : edot(c, j, c.uh) * c.inv_d0;
      c.ubar[j] = c.w[j] * ((1.0 + lin) + quad(c, j, c.Ch));
    }
    for (int p = 0; p < c.npair; ++p) {
      const int j = c.pair[p];
      c.ubp[p] = c.w[j] * (1.0 + quad(c, j, c.Ch));
      c.ubm[p] = in.rect ? c.w[j] * edot(c, j, ut) : c.w1[j] * edot(c, j, c.uh);
      c.Cp[p] = c.ap * c.ubp[p];
      c.Cm[p] = c.am * c.ubm[p];
      c.Chp[p] = c.ahp * c.ubp[p];
      c.Chm[p] = c.ahm * c.ubm[p];
    }
    c.theta = in.kind == MFD_THETA ? in.theta : 1.0;
    c.th1 = 1.0 - c.theta;
    double sp = 0.0;
    for (int p = 0; p < c.npair; ++p) sp = sp + c.Cp[p];
    c.den = 1.0 + c.th1 * (2.0 * sp);
    c.inv_den = 1.0 / c.den;
  } else if (in.eq == kBurgers) {
    c.theta = in.kind == MFD_THETA ? in.theta : 1.0;
    c.th1 = 1.0 - c.theta;
    c.bh = 0.5 * in.dt / in.dx;
    c.beta_one = in.beta == 1.0;
    c.cbeta = (in.beta - 1.0) * d0;
  } else if (in.eq == kNSE) {
    c.theta = in.kind == MFD_THETA ? in.theta : 1.0;
    c.th1 = 1.0 - c.theta;
    c.rho0 = in.rho0;
    c.he_luo = in.he_luo;
    c.rinv0 = 1.0 / in.rho0;
  } else {
    return MFD_E_ARG;
  }
  return MFD_OK;
}

template <typename T>
KC<T> make_kc(const Consts &c) {
  KC<T> k;
  std::memset(&k, 0, sizeof(k));
  for (int j = 0; j < kMaxQ; ++j) {
    k.w[j] = (T)c.w[j];
    k.w1[j] = (T)c.w1[j];
    k.ubar[j] = (T)c.ubar[j];
    for (int a = 0; a < 3; ++a) {
      k.qd[j][a] = (T)c.qd[j][a];
      k.qo[j][a] = (T)c.qo[j][a];
    }
  }
  k.inv_d0 = (T)c.inv_d0;
  k.ap = (T)c.ap; k.am = (T)c.am; k.ahp = (T)c.ahp; k.ahm = (T)c.ahm;
  k.abp = (T)c.abp; k.abm = (T)c.abm; k.abhp = (T)c.abhp; k.abhm = (T)c.abhm;
  for (int i = 0; i < 3; ++i) {
    k.a[i] = (T)c.a[i];
    k.ah[i] = (T)c.ah[i];
  }
  for (int p = 0; p < kMaxP; ++p) {
    k.Cp[p] = (T)c.Cp[p];
    k.Cm[p] = (T)c.Cm[p];
    k.Chp[p] = (T)c.Chp[p];
    k.Chm[p] = (T)c.Chm[p];
    k.Ap[p] = (T)(c.Cp[p] + c.Cm[p]);
    k.Am[p] = (T)(c.Cp[p] - c.Cm[p]);
    k.Ahp[p] = (T)(c.Chp[p] + c.Chm[p]);
    k.Ahm[p] = (T)(c.Chp[p] - c.Chm[p]);
  }
  for (int p = 0; p < c.npair && p < kMaxP; ++p) {
    const int j = c.pair[p];
    k.nw[p][0] = (T)(c.ap * c.w[j]);
    k.nw[p][1] = (T)(c.am * c.w1[j]);
    k.nw[p][2] = (T)(c.abp * c.w1[j]);
    k.nw[p][3] = (T)(c.abm * c.w[j]);
  }
  k.bh = (T)c.bh;
  k.cbeta = (T)c.cbeta;
  k.rho0 = (T)c.rho0;
  k.rinv0 = (T)c.rinv0;
  k.A0 = c.A0; k.Ah0 = c.Ah0; k.Ab0 = c.Ab0; k.Abh0 = c.Abh0;
  k.A0t = (T)c.A0; k.Ah0t = (T)c.Ah0; k.Ab0t = (T)c.Ab0; k.Abh0t = (T)c.Abh0;
  k.th = (T)c.theta;
  k.th1 = (T)c.th1;
  k.inv_den = (T)c.inv_den;
  k.beta_one = c.beta_one;
  k.he_luo = c.he_luo;
  return k;
}

template KC<float> make_kc<float>(const Consts &);
template KC<double> make_kc<double>(const Consts &);

// --------------------------------------------------------------- stability

// Theorem 1, conditions (a)-(c), summed over all j >= 1 (each opposite pair
// twice).  Corollary 2 for three-level schemes of the TRT form.
bool stability_proven(const Consts &c) {
  if (c.eq != kLCDE) return true;  // nonlinear: no sufficient condition checked here
  if (!c.three && c.theta <= 0.5) {
    // Theorem 2 (1): with condition (a) of Theorem 1, A <= 0 and |lambda| <= 1
    for (int p = 0; p < c.npair; ++p)
      if (!(c.ap * c.ubp[p] > 0.0)) return false;
    return true;
  }
  if (!c.three) {
    double sb = 0.0, sc = 0.0;
    for (int p = 0; p < c.npair; ++p) {
      const double t = c.ap * c.ubp[p];
      if (!(t > 0.0)) return false;
      sb += 2.0 * t;
      const double m = c.am * c.ubm[p];
      sc += 2.0 * m * m / t;
    }
    return sb <= 1.0 + 1e-12 && sc <= 1.0 + 1e-12;
  }
  // Corollary 2 (TRT with s+ + s- = 2): ubar+_0 >= 0, ubar+_j > 0,
  // sum (ubar-_j)^2 / ubar+_j <= 1.
  double ub0 = 1.0, sc = 0.0;
  for (int p = 0; p < c.npair; ++p) {
    if (!(c.ubp[p] > 0.0)) return false;
    ub0 -= 2.0 * c.ubp[p];
    sc += 2.0 * c.ubm[p] * c.ubm[p] / c.ubp[p];
  }
  return ub0 >= -1e-12 && sc <= 1.0 + 1e-12;
}

// max over grid modes xi_a = 2 pi m_a / n_a of the largest root modulus.
double max_amplification(const Consts &c, const int64_t n[3]) {
  using cd = std::complex<double>;
  const int64_t nx = n[0], ny = c.dim > 1 ? n[1] : 1, nz = c.dim > 2 ? n[2] : 1;
  double best = 0.0;
  const double tp = 2.0 * M_PI;
  for (int64_t mz = 0; mz < nz; ++mz)
    for (int64_t my = 0; my < ny; ++my)
      for (int64_t mx = 0; mx < nx; ++mx) {
        const double xi[3] = {tp * mx / nx, tp * my / ny, tp * mz / nz};
        cd A1(c.A0, 0.0), A2(c.Ah0, 0.0), z(0.0, 0.0);
        for (int p = 0; p < c.npair; ++p) {
          const int j = c.pair[p];
          double ph = 0.0;
          for (int a = 0; a < c.dim; ++a) ph += c.e[j][a] * xi[a];
          const double cm1 = std::cos(ph) - 1.0, sn = std::sin(ph);
          A1 += 2.0 * cd(c.ap * c.ubp[p] * cm1, c.am * c.ubm[p] * sn);
          A2 += 2.0 * cd(c.ahp * c.ubp[p] * cm1, c.ahm * c.ubm[p] * sn);
          z += 2.0 * cd(c.ap * c.ubp[p] * cm1, c.am * c.ubm[p] * sn);
        }
        double r;
        if (c.theta != 1.0 && !c.three) {
          // Eq. (Tcond1-1), with sum_k a_k = A0
          r = std::abs((c.A0 + c.theta * z) / (1.0 - c.th1 * z));
        } else if (!c.three) {
          r = std::abs(A1);
        } else {
          const cd disc = std::sqrt(A1 * A1 + 4.0 * A2);
          r = std::max(std::abs((A1 + disc) * 0.5), std::abs((A1 - disc) * 0.5));
        }
        best = std::max(best, r);
      }
  return best;
}

// Largest stable time step of the two-level m = 1 family with the linear EDF
// (D0 = I, beta = 1, lambda_bar = 0) and the coefficients of Eq. (LMMFD-2-2):
// a_0 = 1 - s, a_{+-1} = (s -+ 1)/2 with s = 2 alpha dt / (d0 dx^2), so
// ubar+_j = w_j and ubar-_j = w_j e_j.u dt / (d0 dx).
//  * sufficient: Eq. (LMMFD-2-3), |u|^2 <= 2 alpha / dt <= c_s^2 / (1 - w0)
//    with c_s^2 = d0 dx^2 / dt^2;
//  * exact: for a grid mode xi the factor of Eq. (TforMMFD-3) is
//    lambda = 1 - kappa dt X - i dt Y, X = sum_j w_j (1 - cos xi_j) >= 0,
//    Y = sum_j w_j (e_j.u / (d0 dx)) sin xi_j, kappa = 2 alpha / (d0 dx^2);
//    |lambda| <= 1 holds exactly for dt <= 2 kappa X / (kappa^2 X^2 + Y^2),
//    so the bound over the periodic grid's modes is the smallest such dt
//    (modes with X = 0 have lambda = 1).
int max_stable_dt(int lattice, double d0, double dx, const double u[3], double alpha,
                  const int64_t *n, double *dt_suff, double *dt_exact) {
  Consts c;
  std::memset(&c, 0, sizeof(c));
  if (lattice_weights(lattice, d0, c) != 0) return -1;
  double u2 = 0.0;
  for (int a = 0; a < c.dim; ++a) u2 += u[a] * u[a];
  const double t1 = d0 * dx * dx / (2.0 * alpha * (1.0 - c.w[0]));
  *dt_suff = u2 == 0.0 ? t1 : std::min(t1, 2.0 * alpha / u2);
  if (!n || !dt_exact) return 0;
  const int64_t nx = n[0], ny = c.dim > 1 ? n[1] : 1, nz = c.dim > 2 ? n[2] : 1;
  const double kappa = 2.0 * alpha / (d0 * dx * dx);
  const double tp = 2.0 * M_PI;
  double best = HUGE_VAL;
  for (int64_t mz = 0; mz < nz; ++mz)
    for (int64_t my = 0; my < ny; ++my)
      for (int64_t mx = 0; mx < nx; ++mx) {
        const double xi[3] = {tp * mx / nx, tp * my / ny, tp * mz / nz};
        double X = 0.0, Y = 0.0;
        for (int j = 1; j < c.q; ++j) {
          double ph = 0.0, eu = 0.0;
          for (int a = 0; a < c.dim; ++a) {
            ph += c.e[j][a] * xi[a];
            eu += c.e[j][a] * u[a];
          }
          X += c.w[j] * (1.0 - std::cos(ph));
          Y += c.w[j] * eu / (d0 * dx) * std::sin(ph);
        }
        if (X <= 1e-300) continue;
        best = std::min(best, 2.0 * kappa * X / (kappa * kappa * X * X + Y * Y));
      }
  *dt_exact = best;
  return 0;
}

}  // namespace mfd

// ===================================================== C ABI: host algebra

extern "C" int mfd_coeff_moments(const double a[3], const double ah[3], double out[6]) {
  if (!a || !ah || !out) return MFD_E_ARG;
  const double sa = a[0] + a[1] + a[2], sh = ah[0] + ah[1] + ah[2];
  // Eq. (4-2-00a)
  out[0] = sa + sh;
  out[1] = -sh - 1.0;
  out[2] = a[2] - a[0] + ah[2] - ah[0];
  out[3] = 0.5 * (sh - 1.0);
  out[4] = -(ah[2] - ah[0]);
  out[5] = 0.5 * (a[2] + a[0] + ah[2] + ah[0]);
  return MFD_OK;
}

extern "C" int mfd_coeffs_from_constraints(double a0, double A10, double A11, double A21,
                                           double A22, double a[3], double ah[3]) {
  if (!a || !ah) return MFD_E_ARG;
  // Eq. (X): X = (a_1, a_-1, ah_0, ah_1, ah_-1) = A^-1 (1-a0, 1+A10, A11, A21, A22)
  const double a1 = 0.5 * (-a0 + A10 + A11 + A21 + 2.0);
  const double am1 = 0.5 * (-a0 + A10 - A11 - A21 + 2.0);
  const double h0 = 0.5 * (-2.0 * a0 - 4.0 * A22 + 2.0);
  const double h1 = 0.5 * (a0 - A10 - A21 + 2.0 * A22 - 2.0);
  const double hm1 = 0.5 * (a0 - A10 + A21 + 2.0 * A22 - 2.0);
  a[0] = am1; a[1] = a0; a[2] = a1;
  ah[0] = hm1; ah[1] = h0; ah[2] = h1;
  return MFD_OK;
}

extern "C" int mfd_preset(int preset, double param, double a[3], double ah[3]) {
  if (!a || !ah) return MFD_E_ARG;
  for (int i = 0; i < 3; ++i) a[i] = ah[i] = 0.0;
  switch (preset) {
    case MFD_PRESET_SRT:
      a[0] = 1.0;
      return MFD_OK;
    case MFD_PRESET_TRT:  // a_0 = 0, a_1 = 1 - s, a_-1 = 1, ah_0 = -(1 - s)
      a[0] = 1.0;
      a[2] = 1.0 - param;
      ah[1] = -(1.0 - param);
      return MFD_OK;
    case MFD_PRESET_ONE_STAGE:  // a_0 = 2(1 - tau), a_1 = tau - 1, a_-1 = tau
      a[0] = param;
      a[1] = 2.0 * (1.0 - param);
      a[2] = param - 1.0;
      return MFD_OK;
    case MFD_PRESET_TWO_LEVEL:  // Eq. (LMMFD-2-2)
      a[0] = (param + 1.0) / 2.0;
      a[1] = 1.0 - param;
      a[2] = (param - 1.0) / 2.0;
      return MFD_OK;
    default:
      return MFD_E_ARG;
  }
}

extern "C" int mfd_transport_coefficient(const double a[3], const double ah[3], double dx,
                                         double dt, double d0, double beta, double *out) {
  if (!a || !ah || !out || !(dx > 0) || !(dt > 0) || !(d0 > 0)) return MFD_E_ARG;
  double m[6];
  mfd_coeff_moments(a, ah, m);
  if (m[1] == 0.0) return MFD_E_ARG;
  const double cs2 = d0 * (dx / dt) * (dx / dt);
  *out = -(m[5] / m[1]) * dt * beta * cs2;
  return MFD_OK;
}

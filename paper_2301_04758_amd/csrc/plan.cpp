// Host-side sweep plan (see plan.h).
//
// Reference tables: Gauss-Lobatto nodes (roots of P_p' by Newton iteration,
// endpoints added) and the Gauss-Legendre rule (roots of P_nq by Newton), both
// mirrored so that z[k-i] == 1 - z[i] holds exactly; Lagrange polynomials in
// barycentric form.  Geometry: the element map of Sec. 3.1 and its Jacobian
// F (Sec. 3.2) at every quadrature point; adj(F) = J F^{-1} carries the
// reference-space streaming term, n ds the face terms.  Upwind masks follow the
// chord rule stated in vef_sweep.h; levels come from Kahn's algorithm.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>

namespace vefplan {

namespace {

// P_k(x) and P_k'(x) on [-1, 1] (Bonnet recurrence).
void legendre_pair(int k, double x, double &pk, double &dk) {
  double a = 1.0, b = x;  // P_0, P_1
  if (k == 0) {
    pk = 1.0;
    dk = 0.0;
    return;
  }
  for (int j = 1; j < k; ++j) {
    double c = ((2 * j + 1) * x * b - j * a) / (j + 1);
    a = b;
    b = c;
  }
  pk = b;
  dk = k * (a - x * b) / (1.0 - x * x);
}

// Second derivative of P_k from the Legendre ODE.
double legendre_d2(int k, double x, double pk, double dk) {
  return (2.0 * x * dk - k * (k + 1.0) * pk) / (1.0 - x * x);
}

void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    // i-th largest root on [-1,1], Tricomi-type initial guess
    double t = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
    double pk = 0, dk = 1;
    for (int it = 0; it < 60; ++it) {
      legendre_pair(n, t, pk, dk);
      double step = pk / dk;
      t -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    legendre_pair(n, t, pk, dk);
    double wt = 2.0 / ((1.0 - t * t) * dk * dk);
    // t is the i-th largest root: position n-1-i on [0,1], mirrored at i
    double hi = 0.5 * (1.0 + t);
    x[n - 1 - i] = hi;
    x[i] = 1.0 - hi;
    w[n - 1 - i] = 0.5 * wt;
    w[i] = 0.5 * wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.5;
}

void gauss_lobatto01(int k, std::vector<double> &z) {
  z.assign(k + 1, 0.0);
  z[0] = 0.0;
  z[k] = 1.0;
  // interior nodes: roots of P_k' on (-1, 1), Newton on P_k' using P_k''
  for (int i = 1; i <= k / 2; ++i) {
    double t = std::cos(M_PI * i / k);  // Chebyshev-Gauss-Lobatto guess, descending
    for (int it = 0; it < 60; ++it) {
      double pk, dk;
      legendre_pair(k, t, pk, dk);
      double d2 = legendre_d2(k, t, pk, dk);
      double step = dk / d2;
      t -= step;
      if (std::fabs(step) <= 1e-17) break;
    }
    double hi = 0.5 * (1.0 + t);
    z[k - i] = hi;
    z[i] = 1.0 - hi;
  }
  if (k % 2 == 0) z[k / 2] = 0.5;
}

// Barycentric Lagrange interpolation on nodes z: values and derivatives of all
// basis polynomials at x.
void bary_eval(const std::vector<double> &z, double x, double *val, double *der) {
  const int k = (int)z.size();
  double bw[kMaxP + kMaxM + 2];
  for (int j = 0; j < k; ++j) {
    double prod = 1.0;
    for (int l = 0; l < k; ++l)
      if (l != j) prod *= (z[j] - z[l]);
    bw[j] = 1.0 / prod;
  }
  for (int j = 0; j < k; ++j) {
    if (x == z[j]) {
      // at a node: value delta_jl, derivative from the differentiation matrix
      for (int l = 0; l < k; ++l) val[l] = (l == j) ? 1.0 : 0.0;
      if (der) {
        double djj = 0.0;
        for (int l = 0; l < k; ++l) {
          if (l == j) continue;
          der[l] = (bw[l] / bw[j]) / (z[j] - z[l]);
          djj -= der[l];
        }
        der[j] = djj;
      }
      return;
    }
  }
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += bw[j] / (x - z[j]);
  for (int j = 0; j < k; ++j) val[j] = (bw[j] / (x - z[j])) / s;
  if (der) {
    // l_j'(x) = l_j(x) * sum_{m != j} 1/(x - z_m)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int l = 0; l < k; ++l)
        if (l != j) acc += 1.0 / (x - z[l]);
      der[j] = val[j] * acc;
    }
  }
}

// Face f of the reference square at parameter s (counter-clockwise).
inline void face_ref(int f, double s, double &xi, double &eta) {
  switch (f) {
    case 0: xi = s; eta = 0.0; break;
    case 1: xi = 1.0; eta = s; break;
    case 2: xi = 1.0 - s; eta = 1.0; break;
    default: xi = 0.0; eta = 1.0 - s; break;
  }
}

struct GeomEval {
  int m;
  std::vector<double> z;  // geometry nodes
  // x, F at (xi, eta) for control points X[(m+1)^2][2]
  void eval(const double *X, double xi, double eta, double *x, double F[2][2]) const {
    double vx[kMaxM + 1], dx[kMaxM + 1], vy[kMaxM + 1], dy[kMaxM + 1];
    bary_eval(z, xi, vx, dx);
    bary_eval(z, eta, vy, dy);
    double px = 0, py = 0, f00 = 0, f01 = 0, f10 = 0, f11 = 0;
    for (int b = 0; b <= m; ++b)
      for (int a = 0; a <= m; ++a) {
        const double *c = X + 2 * (a + (m + 1) * b);
        double v = vx[a] * vy[b], gx = dx[a] * vy[b], gy = vx[a] * dy[b];
        px += c[0] * v;
        py += c[1] * v;
        f00 += c[0] * gx;
        f01 += c[0] * gy;
        f10 += c[1] * gx;
        f11 += c[1] * gy;
      }
    if (x) {
      x[0] = px;
      x[1] = py;
    }
    F[0][0] = f00;
    F[0][1] = f01;
    F[1][0] = f10;
    F[1][1] = f11;
  }
};

inline void corner_pair(int m, int f, int &a, int &b) {
  const int c00 = 0, c10 = m, c01 = m * (m + 1), c11 = (m + 1) * (m + 1) - 1;
  static const int dummy = 0;
  (void)dummy;
  switch (f) {
    case 0: a = c00; b = c10; break;
    case 1: a = c10; b = c11; break;
    case 2: a = c11; b = c01; break;
    default: a = c01; b = c00; break;
  }
}

int fail(std::string &err, int code, const char *fmt, long long a = 0, long long b = 0) {
  char buf[256];
  std::snprintf(buf, sizeof(buf), fmt, a, b);
  err = buf;
  return code;
}

}  // namespace

int build_tables(int p, int nq, Tables &t) {
  if (p < 1 || p > kMaxP || nq < 1 || nq > kMaxP + kMaxM + 1) return VEF_ERR_INVALID;
  t.p = p;
  t.nq = nq;
  gauss_lobatto01(p, t.gl);
  gauss_legendre01(nq, t.gx, t.gw);
  const int P1 = p + 1, n = P1 * P1, Q = nq * nq;
  std::vector<double> v1(nq * P1), d1(nq * P1);
  for (int q = 0; q < nq; ++q) bary_eval(t.gl, t.gx[q], &v1[q * P1], &d1[q * P1]);
  t.V.assign(Q * n, 0.0);
  t.Dx.assign(Q * n, 0.0);
  t.Dy.assign(Q * n, 0.0);
  for (int qy = 0; qy < nq; ++qy)
    for (int qx = 0; qx < nq; ++qx) {
      const int q = qx + nq * qy;
      for (int b = 0; b < P1; ++b)
        for (int a = 0; a < P1; ++a) {
          const int i = a + P1 * b;
          t.V[q * n + i] = v1[qx * P1 + a] * v1[qy * P1 + b];
          t.Dx[q * n + i] = d1[qx * P1 + a] * v1[qy * P1 + b];
          t.Dy[q * n + i] = v1[qx * P1 + a] * d1[qy * P1 + b];
        }
    }
  t.F = v1;
  // affine-element tables (quadrature sums with the same rule)
  t.affine.assign(3 * n * n + P1 * P1 + Q * n + nq * P1 + P1 * P1, 0.0);
  double *Mt = t.affine.data(), *Gx = Mt + n * n, *Gy = Gx + n * n, *M1 = Gy + n * n;
  double *WV = M1 + P1 * P1, *WL = WV + Q * n, *GD1 = WL + nq * P1;
  for (int q = 0; q < Q; ++q) {
    const double w = t.gw[q % nq] * t.gw[q / nq];
    for (int i = 0; i < n; ++i) {
      WV[q * n + i] = w * t.V[q * n + i];
      for (int j = 0; j < n; ++j) {
        Mt[j * n + i] += w * t.V[q * n + i] * t.V[q * n + j];
        Gx[j * n + i] += w * t.Dx[q * n + i] * t.V[q * n + j];
        Gy[j * n + i] += w * t.Dy[q * n + i] * t.V[q * n + j];
      }
    }
  }
  for (int q = 0; q < nq; ++q)
    for (int a = 0; a < P1; ++a) {
      WL[q * P1 + a] = t.gw[q] * v1[q * P1 + a];
      for (int c = 0; c < P1; ++c) {
        M1[a * P1 + c] += t.gw[q] * v1[q * P1 + a] * v1[q * P1 + c];
        // 1D factors of the tensor-product matrices: Mt = M1 (x) M1,
        // Gx = GD1 (x) M1, Gy = M1 (x) GD1 (test index first)
        GD1[a * P1 + c] += t.gw[q] * d1[q * P1 + a] * v1[q * P1 + c];
      }
    }
  return VEF_OK;
}

int hrt_sizes(int p, int nq, HrtSizes &z) {
  if (p < 1 || p > 3 || nq < p + 2 || nq > p + 3) return VEF_ERR_INVALID;
  z.p = p;
  z.nq = nq;
  z.nx = (p + 2) * (p + 1);
  z.nv = 2 * z.nx;
  z.nphi = (p + 1) * (p + 1);
  z.nt = (p + 1) * (p + 1);
  const int Q = nq * nq;
  z.off_w = 0;
  z.off_vr = z.off_w + Q;
  z.off_dr = z.off_vr + Q * z.nv;
  z.off_u = z.off_dr + 2 * Q * z.nv;
  z.off_tv = z.off_u + Q * z.nphi;
  z.off_vrf = z.off_tv + Q * z.nt;
  z.off_tf = z.off_vrf + 4 * nq * z.nv;
  z.off_wf = z.off_tf + 4 * nq * z.nt;
  z.off_mv = z.off_wf + nq;               // [nv][nv] sum_q w vr_i vr_j
  z.off_dv = z.off_mv + z.nv * z.nv;      // [nphi][nv] sum_q w u_i div vr_j
  z.off_mu = z.off_dv + z.nphi * z.nv;    // [nphi][nphi] sum_q w u_i u_j
  z.off_lf = z.off_mu + z.nphi * z.nphi;  // [nq][p+1] face multiplier basis at the Gauss points
  z.off_lr = z.off_lf + nq * (p + 1);     // [nq][p+1] the same at 1 - (Gauss points)
  z.total = z.off_lr + nq * (p + 1);
  return VEF_OK;
}

int build_hrt_tables(int p, int nq, std::vector<double> &blob) {
  HrtSizes z;
  if (hrt_sizes(p, nq, z)) return VEF_ERR_INVALID;
  std::vector<double> lob1, lob, gx, gw, leg, lw;
  gauss_lobatto01(p + 1, lob1);  // RT normal direction: degree p + 1, closed points
  gauss_lobatto01(p, lob);       // transport basis: degree p, closed points
  gauss_legendre01(nq, gx, gw);  // quadrature
  gauss_legendre01(p + 1, leg, lw);  // RT tangential direction and phi: p + 1 open points
  const int Q = nq * nq;
  blob.assign(z.total, 0.0);
  // 1D values and derivatives at a point
  auto eval = [](const std::vector<double> &nodes, double x, std::vector<double> &v, std::vector<double> &d) {
    v.assign(nodes.size(), 0.0);
    d.assign(nodes.size(), 0.0);
    bary_eval(nodes, x, v.data(), d.data());
  };
  // one RT function's non-zero component and its (xi, eta) derivatives at (x, y)
  std::vector<double> L1x, dL1x, L1y, dL1y, Gx, dGx, Gy, dGy, Tx, dTx, Ty, dTy;
  auto rt_at = [&](double x, double y, double *val, double *dval) {
    eval(lob1, x, L1x, dL1x);
    eval(lob1, y, L1y, dL1y);
    eval(leg, x, Gx, dGx);
    eval(leg, y, Gy, dGy);
    int i = 0;
    for (int b = 0; b <= p; ++b)
      for (int a = 0; a <= p + 1; ++a, ++i) {  // xi component
        val[i] = L1x[a] * Gy[b];
        if (dval) {
          dval[2 * i] = dL1x[a] * Gy[b];
          dval[2 * i + 1] = L1x[a] * dGy[b];
        }
      }
    for (int b = 0; b <= p + 1; ++b)
      for (int a = 0; a <= p; ++a, ++i) {  // eta component
        val[i] = Gx[a] * L1y[b];
        if (dval) {
          dval[2 * i] = dGx[a] * L1y[b];
          dval[2 * i + 1] = Gx[a] * dL1y[b];
        }
      }
  };
  auto tensor = [&](const std::vector<double> &nodes, double x, double y, double *out) {
    eval(nodes, x, Tx, dTx);
    eval(nodes, y, Ty, dTy);
    const int k = (int)nodes.size();
    for (int b = 0; b < k; ++b)
      for (int a = 0; a < k; ++a) out[a + k * b] = Tx[a] * Ty[b];
  };
  for (int qy = 0; qy < nq; ++qy)
    for (int qx = 0; qx < nq; ++qx) {
      const int q = qx + nq * qy;
      const double x = gx[qx], y = gx[qy];
      blob[z.off_w + q] = gw[qx] * gw[qy];
      rt_at(x, y, &blob[z.off_vr + (size_t)q * z.nv], &blob[z.off_dr + (size_t)q * z.nv * 2]);
      tensor(leg, x, y, &blob[z.off_u + (size_t)q * z.nphi]);
      tensor(lob, x, y, &blob[z.off_tv + (size_t)q * z.nt]);
    }
  for (int f = 0; f < 4; ++f)
    for (int q = 0; q < nq; ++q) {
      const double s = gx[q];
      double x, y;  // counter-clockwise face parameter
      switch (f) {
        case 0: x = s; y = 0.0; break;
        case 1: x = 1.0; y = s; break;
        case 2: x = 1.0 - s; y = 1.0; break;
        default: x = 0.0; y = 1.0 - s; break;
      }
      rt_at(x, y, &blob[z.off_vrf + ((size_t)f * nq + q) * z.nv], nullptr);
      tensor(lob, x, y, &blob[z.off_tf + ((size_t)f * nq + q) * z.nt]);
    }
  for (int q = 0; q < nq; ++q) blob[z.off_wf + q] = gw[q];
  // The interior-face multiplier: Lagrange of degree p through the
  // Gauss-Legendre points of the face, in the counter-clockwise parameter of
  // the face's lower-numbered element (its other element sees 1 - s).
  {
    std::vector<double> v, dv;
    for (int q = 0; q < nq; ++q) {
      eval(leg, gx[q], v, dv);
      for (int t = 0; t <= p; ++t) blob[z.off_lf + (size_t)q * (p + 1) + t] = v[t];
      eval(leg, 1.0 - gx[q], v, dv);
      for (int t = 0; t <= p; ++t) blob[z.off_lr + (size_t)q * (p + 1) + t] = v[t];
    }
  }
  // Reference matrices of the element-independent parts of the affine
  // blocks: the RT mass of the non-zero components (A = sigma_t / J
  // (F^T F)_{c_i c_j} times it), D, and the Q_p mass (Ma = sigma_a J times it).
  for (int q = 0; q < Q; ++q) {
    const double w = blob[z.off_w + q];
    const double *vr = &blob[z.off_vr + (size_t)q * z.nv];
    const double *dr = &blob[z.off_dr + (size_t)q * z.nv * 2];
    const double *u = &blob[z.off_u + (size_t)q * z.nphi];
    for (int i = 0; i < z.nv; ++i)
      for (int j = 0; j < z.nv; ++j) blob[z.off_mv + (size_t)i * z.nv + j] += w * vr[i] * vr[j];
    for (int i = 0; i < z.nphi; ++i)
      for (int j = 0; j < z.nv; ++j)
        blob[z.off_dv + (size_t)i * z.nv + j] += w * u[i] * dr[2 * j + (j < z.nx ? 0 : 1)];
    for (int i = 0; i < z.nphi; ++i)
      for (int j = 0; j < z.nphi; ++j) blob[z.off_mu + (size_t)i * z.nphi + j] += w * u[i] * u[j];
  }
  return VEF_OK;
}

int build_problem_plan(const vef_problem_desc &d, bool lag_cycles, bool pointwise, ProblemPlan &o,
                       std::string &err) {
  if (d.p < 1 || d.p > kMaxP) return fail(err, VEF_ERR_INVALID, "p=%lld out of range 1..4", d.p);
  if (d.m < 1 || d.m > kMaxM) return fail(err, VEF_ERR_INVALID, "m=%lld out of range 1..3", d.m);
  const int nq = d.nq > 0 ? d.nq : d.p + d.m;
  if (nq < d.p + 1 || nq > d.p + 3)
    return fail(err, VEF_ERR_INVALID, "nq=%lld outside p+1..p+3 (p=%lld)", nq, d.p);
  if (d.n_elem < 1 || d.n_cp < 4) return fail(err, VEF_ERR_INVALID, "n_elem=%lld n_cp=%lld", d.n_elem, d.n_cp);
  if (d.n_elem > (1 << 22)) return fail(err, VEF_ERR_INVALID, "n_elem=%lld too large (max 4194304)", d.n_elem);
  if (d.n_dir < 1 || d.n_dir > kMaxDirs) return fail(err, VEF_ERR_INVALID, "n_dir=%lld out of range 1..1024", d.n_dir);
  if (!d.cp_xy || !d.elem_cp || !d.omega || !d.weight || !d.sigma_t || !d.sigma_s)
    return fail(err, VEF_ERR_INVALID, "NULL array in problem description");
  const int m = d.m, ncp_e = (m + 1) * (m + 1), ne = d.n_elem, nd = d.n_dir;
  for (long long i = 0; i < (long long)ne * ncp_e; ++i)
    if (d.elem_cp[i] < 0 || d.elem_cp[i] >= d.n_cp)
      return fail(err, VEF_ERR_INVALID, "elem_cp[%lld]=%lld out of range", i, d.elem_cp[i]);
  for (long long i = 0; i < 2LL * d.n_cp; ++i)
    if (!std::isfinite(d.cp_xy[i])) return fail(err, VEF_ERR_INVALID, "cp_xy[%lld] not finite", i);
  double wsum = 0.0;
  for (int k = 0; k < nd; ++k) {
    const double ox = d.omega[2 * k], oy = d.omega[2 * k + 1], w = d.weight[k];
    if (!std::isfinite(ox) || !std::isfinite(oy) || ox * ox + oy * oy > 1.0 + 1e-12)
      return fail(err, VEF_ERR_INVALID, "direction %lld not a unit-sphere projection", k);
    if (!(w > 0.0) || !std::isfinite(w)) return fail(err, VEF_ERR_INVALID, "weight %lld not positive", k);
    wsum += w;
  }
  if (std::fabs(wsum - 4.0 * M_PI) > 1e-12 * 4.0 * M_PI)
    return fail(err, VEF_ERR_INVALID, "angular weights must sum to 4 pi");
  for (int e = 0; e < ne; ++e)
    if (!(d.sigma_t[e] >= 0.0) || !(d.sigma_s[e] >= 0.0) || !std::isfinite(d.sigma_t[e]) ||
        !std::isfinite(d.sigma_s[e]))
      return fail(err, VEF_ERR_INVALID, "cross sections of element %lld not finite and >= 0", e);

  o.p = d.p;
  o.m = m;
  o.nq = nq;
  o.n = (d.p + 1) * (d.p + 1);
  o.Q = nq * nq;
  o.ne = ne;
  o.nd = nd;
  int rc = build_tables(d.p, nq, o.tab);
  if (rc) return fail(err, rc, "tables p=%lld nq=%lld", d.p, nq);
  const Tables &T = o.tab;

  GeomEval G;
  G.m = m;
  gauss_lobatto01(m, G.z);

  // ---- geometry at volume and face points
  o.geo_v.assign((size_t)ne * o.Q * 5, 0.0);
  o.geo_f.assign((size_t)ne * 4 * nq * 2, 0.0);
  std::vector<double> X(2 * ncp_e);
  for (int e = 0; e < ne; ++e) {
    // control points relative to the element's first one: the map derivatives
    // (all that is evaluated here) are unchanged, and the sums no longer
    // cancel coordinates of domain size down to element size
    const double *c0 = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e];
    for (int i = 0; i < ncp_e; ++i) {
      const int c = d.elem_cp[(size_t)e * ncp_e + i];
      X[2 * i] = d.cp_xy[2 * c] - c0[0];
      X[2 * i + 1] = d.cp_xy[2 * c + 1] - c0[1];
    }
    for (int qy = 0; qy < nq; ++qy)
      for (int qx = 0; qx < nq; ++qx) {
        double F[2][2];
        G.eval(X.data(), T.gx[qx], T.gx[qy], nullptr, F);
        const double J = F[0][0] * F[1][1] - F[0][1] * F[1][0];
        if (!(J > 0.0))
          return fail(err, VEF_ERR_JACOBIAN, "element %lld: Jacobian <= 0 at volume point %lld", e, qx + nq * qy);
        const double w = T.gw[qx] * T.gw[qy];
        double *g = &o.geo_v[((size_t)e * o.Q + qx + nq * qy) * 5];
        g[0] = w * J;
        g[1] = w * F[1][1];   // adj(F) = [[y_eta, -x_eta], [-y_xi, x_xi]]
        g[2] = -w * F[0][1];
        g[3] = -w * F[1][0];
        g[4] = w * F[0][0];
      }
    for (int f = 0; f < 4; ++f)
      for (int q = 0; q < nq; ++q) {
        double xi, eta, F[2][2];
        face_ref(f, T.gx[q], xi, eta);
        G.eval(X.data(), xi, eta, nullptr, F);
        double tx, ty;  // dx/ds along the counter-clockwise parameterisation
        switch (f) {
          case 0: tx = F[0][0]; ty = F[1][0]; break;
          case 1: tx = F[0][1]; ty = F[1][1]; break;
          case 2: tx = -F[0][0]; ty = -F[1][0]; break;
          default: tx = -F[0][1]; ty = -F[1][1]; break;
        }
        double *g = &o.geo_f[(((size_t)e * 4 + f) * nq + q) * 2];
        g[0] = T.gw[q] * ty;   // outward n ds = clockwise rotation of the tangent
        g[1] = -T.gw[q] * tx;
      }
  }

  // ---- faces: match by the pair of corner control points
  o.nbr.assign((size_t)ne * 4, -1);
  o.nbr_face.assign((size_t)ne * 4, -1);
  std::unordered_map<uint64_t, int> first;  // key -> 4*e+f
  first.reserve((size_t)ne * 4);
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < 4; ++f) {
      int la, lb;
      corner_pair(m, f, la, lb);
      const uint32_t ga = (uint32_t)d.elem_cp[(size_t)e * ncp_e + la];
      const uint32_t gb = (uint32_t)d.elem_cp[(size_t)e * ncp_e + lb];
      if (ga == gb) return fail(err, VEF_ERR_INVALID, "element %lld face %lld is degenerate", e, f);
      const uint64_t key = ((uint64_t)std::min(ga, gb) << 32) | std::max(ga, gb);
      auto it = first.find(key);
      if (it == first.end()) {
        first.emplace(key, 4 * e + f);
        continue;
      }
      const int o4 = it->second;
      if (o4 < 0) return fail(err, VEF_ERR_INVALID, "face of element %lld shared by more than two elements", e);
      const int e2 = o4 >> 2, f2 = o4 & 3;
      int la2, lb2;
      corner_pair(m, f2, la2, lb2);
      // both elements run counter-clockwise: the shared face must be reversed
      if ((uint32_t)d.elem_cp[(size_t)e2 * ncp_e + la2] != gb)
        return fail(err, VEF_ERR_INVALID, "elements %lld and %lld are not consistently oriented", e, e2);
      o.nbr[4 * e + f] = e2;
      o.nbr_face[4 * e + f] = (int8_t)f2;
      o.nbr[o4] = e;
      o.nbr_face[o4] = (int8_t)f;
      it->second = -1;
    }
  o.bf_ef.clear();
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < 4; ++f)
      if (o.nbr[4 * e + f] < 0) {
        o.nbr[4 * e + f] = -(int)(o.bf_ef.size() + 1);
        o.bf_ef.push_back(4 * e + f);
      }
  o.nbf = (int)o.bf_ef.size();

  // chords N_F = rot(x_end - x_start), exactly antisymmetric between the two sides
  std::vector<double> chord((size_t)ne * 8);
  for (int e = 0; e < ne; ++e)
    for (int f = 0; f < 4; ++f) {
      int la, lb;
      corner_pair(m, f, la, lb);
      const double *xa = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + la];
      const double *xb = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + lb];
      chord[8 * e + 2 * f] = xb[1] - xa[1];
      chord[8 * e + 2 * f + 1] = -(xb[0] - xa[0]);
    }

  // ---- upwind masks per direction; one decision per interior face pair
  // (pointwise: an inflow bit wherever some face point has Omega . n < 0)
  o.mask.assign((size_t)nd * ne, 0);
  for (int k = 0; k < nd; ++k) {
    const double ox = d.omega[2 * k], oy = d.omega[2 * k + 1];
    uint8_t *mk = &o.mask[(size_t)k * ne];
    if (pointwise) {
      for (int e = 0; e < ne; ++e)
        for (int f = 0; f < 4; ++f)
          for (int q = 0; q < nq; ++q) {
            const double *g = &o.geo_f[(((size_t)e * 4 + f) * nq + q) * 2];
            if (ox * g[0] + oy * g[1] < 0.0) {
              mk[e] |= (uint8_t)(1u << f);
              break;
            }
          }
      continue;
    }
    for (int e = 0; e < ne; ++e)
      for (int f = 0; f < 4; ++f) {
        const int nb = o.nbr[4 * e + f];
        const double s = std::fma(ox, chord[8 * e + 2 * f], oy * chord[8 * e + 2 * f + 1]);
        if (nb < 0) {
          if (s < 0.0) mk[e] |= (uint8_t)(1u << f);
          continue;
        }
        if (nb < e) continue;  // decided from the lower element of the pair
        bool self_up = s > 0.0 ? true : (s < 0.0 ? false : true /* e < nb: lower id upwind */);
        const int f2 = o.nbr_face[4 * e + f];
        if (self_up)
          mk[nb] |= (uint8_t)(1u << f2);
        else
          mk[e] |= (uint8_t)(1u << f);
      }
  }

  // ---- direction classes with identical masks
  o.dir_group.assign(nd, -1);
  o.group_rep.clear();
  for (int k = 0; k < nd; ++k) {
    const uint8_t *mk = &o.mask[(size_t)k * ne];
    for (size_t g = 0; g < o.group_rep.size(); ++g) {
      const uint8_t *mg = &o.mask[(size_t)o.group_rep[g] * ne];
      if (std::equal(mk, mk + ne, mg)) {
        o.dir_group[k] = (int)g;
        break;
      }
    }
    if (o.dir_group[k] < 0) {
      o.dir_group[k] = (int)o.group_rep.size();
      o.group_rep.push_back(k);
    }
  }
  o.n_groups = (int)o.group_rep.size();

  // ---- Kahn levels per class
  o.level.assign((size_t)o.n_groups * ne, 0);
  o.order.assign((size_t)o.n_groups * ne, 0);
  o.n_levels_g.assign(o.n_groups, 0);
  o.level_off.clear();
  o.n_levels = 0;
  std::vector<int> indeg(ne), queue(ne);
  std::vector<uint8_t> placed(ne);
  o.lag_mask.assign((size_t)o.n_groups * ne, 0);
  o.n_lagged = 0;
  std::vector<std::vector<int>> offs(o.n_groups);
  for (int g = 0; g < o.n_groups; ++g) {
    const uint8_t *mk = &o.mask[(size_t)o.group_rep[g] * ne];
    int32_t *lev = &o.level[(size_t)g * ne];
    for (int e = 0; e < ne; ++e) {
      int c = 0;
      for (int f = 0; f < 4; ++f)
        if ((mk[e] >> f & 1) && o.nbr[4 * e + f] >= 0) ++c;
      indeg[e] = c;
    }
    uint8_t *lagm = &o.lag_mask[(size_t)g * ne];
    int head = 0, tail = 0, n_lag = 0;
    for (int e = 0; e < ne; ++e)
      if (!indeg[e]) queue[tail++] = e;
    std::fill(placed.begin(), placed.end(), (uint8_t)0);
    for (int t = 0; t < tail; ++t) placed[queue[t]] = 1;
    int maxl = 0;
    for (;;) {
      while (head < tail) {
        const int e = queue[head++];
        maxl = std::max(maxl, (int)lev[e]);
        for (int f = 0; f < 4; ++f) {
          const int nb = o.nbr[4 * e + f];
          if (nb < 0) continue;
          // nb waits on e when its face toward e is an inflow face (with
          // whole-face upwinding exactly when e's face is not; a pointwise
          // face with both signs is an inflow face of both)
          const int f2 = o.nbr_face[4 * e + f];
          if (!(mk[nb] >> f2 & 1) || placed[nb]) continue;  // released elements are placed
          lev[nb] = std::max(lev[nb], lev[e] + 1);
          if (--indeg[nb] == 0) {
            queue[tail++] = nb;
            placed[nb] = 1;
          }
        }
      }
      if (tail == ne) break;
      if (!lag_cycles)
        return fail(err, VEF_ERR_CYCLE, "upwind graph of direction %lld has a cycle (%lld elements left)",
                    o.group_rep[g], ne - tail);
      // Every element left waits on a cycle.  Release the one with the
      // fewest unsolved upwind neighbours (lowest id on ties); its couplings
      // to them are lagged: read from the previous sweep's angular flux.
      int best = -1;
      for (int e = 0; e < ne; ++e)
        if (!placed[e] && (best < 0 || indeg[e] < indeg[best])) best = e;
      for (int f = 0; f < 4; ++f) {
        const int nb = o.nbr[4 * best + f];
        if (nb >= 0 && (mk[best] >> f & 1) && !placed[nb]) {
          lagm[best] |= (uint8_t)(1u << f);
          ++n_lag;
        }
      }
      indeg[best] = 0;
      queue[tail++] = best;
      placed[best] = 1;
    }
    if (n_lag) {
      // Levels of the lagged order: an element follows its non-lagged upwind
      // neighbours, and precedes the elements it reads lagged data from, so
      // that those are overwritten only after the read.  queue holds a
      // topological order of both relations.
      std::fill(lev, lev + ne, 0);
      maxl = 0;
      for (int t = 0; t < ne; ++t) {
        const int e = queue[t];
        maxl = std::max(maxl, (int)lev[e]);
        for (int f = 0; f < 4; ++f) {
          const int nb = o.nbr[4 * e + f];
          if (nb < 0) continue;
          const bool inflow = mk[e] >> f & 1;
          const bool after = inflow ? (lagm[e] >> f & 1) != 0 : !(lagm[nb] >> o.nbr_face[4 * e + f] & 1);
          if (after) lev[nb] = std::max(lev[nb], lev[e] + 1);
        }
      }
      long long nd_g = 0;
      for (int k = 0; k < nd; ++k) nd_g += o.dir_group[k] == g;
      o.n_lagged += nd_g * n_lag;
    }
    o.n_levels_g[g] = maxl + 1;
    o.n_levels = std::max(o.n_levels, maxl + 1);
    // counting sort by level, ties by element id
    std::vector<int> cnt(maxl + 2, 0);
    for (int e = 0; e < ne; ++e) cnt[lev[e] + 1]++;
    for (int l = 0; l <= maxl; ++l) cnt[l + 1] += cnt[l];
    offs[g] = cnt;
    std::vector<int> pos(cnt.begin(), cnt.end() - 1);
    int32_t *ord = &o.order[(size_t)g * ne];
    for (int e = 0; e < ne; ++e) ord[pos[lev[e]]++] = e;
  }
  o.level_off.assign((size_t)o.n_groups * (o.n_levels + 1), 0);
  for (int g = 0; g < o.n_groups; ++g)
    for (int l = 0; l <= o.n_levels; ++l)
      o.level_off[(size_t)g * (o.n_levels + 1) + l] = offs[g][std::min(l, (int)offs[g].size() - 1)];

  // packed element descriptors in (level, id) order per class
  o.desc_ef.assign((size_t)o.n_groups * ne * 2, 0);
  o.desc_nb.assign((size_t)o.n_groups * ne * 4, 0);
  o.desc_up.assign((size_t)o.n_groups * ne * 4, 0u);
  o.max_width = 1;
  o.max_gap = 0;
  std::vector<int> pos_in_level(ne);
  for (int g = 0; g < o.n_groups; ++g) {
    const uint8_t *mk = &o.mask[(size_t)o.group_rep[g] * ne];
    const int32_t *ord = &o.order[(size_t)g * ne];
    const int32_t *lev = &o.level[(size_t)g * ne];
    const uint8_t *lagm_g = &o.lag_mask[(size_t)g * ne];
    const int *lo = &o.level_off[(size_t)g * (o.n_levels + 1)];
    for (int t = 0; t < ne; ++t) pos_in_level[ord[t]] = t - lo[lev[ord[t]]];
    for (int t = 0; t < ne; ++t) {
      const int e = ord[t];
      int flags = mk[e];
      for (int f = 0; f < 4; ++f) {
        flags |= (std::max<int>(o.nbr_face[4 * e + f], 0) & 3) << (4 + 2 * f);
        const int nb = o.nbr[4 * e + f];
        o.desc_nb[((size_t)g * ne + t) * 4 + f] = nb;
        if (nb >= 0 && ((mk[e] >> f) & 1)) {
          const bool lagged = lagm_g[e] >> f & 1;
          const int gap = lagged ? 255 : lev[e] - lev[nb];
          if (!lagged) o.max_gap = std::max(o.max_gap, gap);
          const uint32_t code = (uint32_t)std::min(gap, 255) | ((uint32_t)pos_in_level[nb] << 8) |
                                ((uint32_t)(o.nbr_face[4 * e + f] & 3) << 30);
          o.desc_up[((size_t)g * ne + t) * 4 + f] = code;
        }
      }
      o.desc_ef[((size_t)g * ne + t) * 2] = e;
      o.desc_ef[((size_t)g * ne + t) * 2 + 1] = flags;
    }
    for (int L = 0; L < o.n_levels; ++L) {
      const int *lo = &o.level_off[(size_t)g * (o.n_levels + 1)];
      o.max_width = std::max(o.max_width, lo[L + 1] - lo[L]);
    }
  }

  // straight faces: every control point of a face on the chord of its corners
  // (to the rounding of the coordinates, whose size R bounds the error of
  // the cross product together with the chord length)
  o.straight = true;
  const double eps_geo = 256.0 * 2.220446049250313e-16;
  for (int e = 0; e < ne && o.straight && m > 1; ++e)
    for (int f = 0; f < 4 && o.straight; ++f) {
      int la, lb;
      corner_pair(m, f, la, lb);
      const double *xa = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + la];
      const double *xb = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + lb];
      const double cx = xb[0] - xa[0], cy = xb[1] - xa[1];
      for (int k = 1; k < m; ++k) {
        int li;
        switch (f) {
          case 0: li = k; break;
          case 1: li = m + (m + 1) * k; break;
          case 2: li = k + (m + 1) * m; break;
          default: li = (m + 1) * k; break;
        }
        const double *xi = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + li];
        const double cr = (xi[0] - xa[0]) * cy - (xi[1] - xa[1]) * cx;
        const double R = std::max(std::max(std::fabs(xa[0]), std::fabs(xa[1])),
                                  std::max(std::fabs(xi[0]), std::fabs(xi[1])));
        const double c2 = cx * cx + cy * cy;
        if (std::fabs(cr) > 1e-13 * c2 + eps_geo * R * std::sqrt(c2)) o.straight = false;
      }
    }
  double smin = d.sigma_t[0];
  for (int e = 1; e < ne; ++e) smin = std::min(smin, d.sigma_t[e]);
  o.nopivot = o.straight && smin > 0.0;

  // Per (direction, element), bit 7 of the mask: the local matrix is not
  // certified for elimination in natural order.  It is certified when
  // sigma_t > 0 and Omega . n has the sign of the face's role at every face
  // quadrature point (>= 0 on outflow faces, <= 0 on inflow faces): with the
  // exact quadrature of the reading, u^T A u = int sigma_t u^2 +
  // 1/2 sum_f int_f |Omega . n| u^2 > 0, so every leading block of A is
  // non-singular.  Straight faces always qualify; curved faces whose normal
  // turns through Omega do not.  Set after the direction classes, which
  // depend on the inflow bits only.
  if (!o.nopivot) {
    for (int k = 0; k < nd; ++k) {
      const double ox = d.omega[2 * k], oy = d.omega[2 * k + 1];
      uint8_t *mk = &o.mask[(size_t)k * ne];
      for (int e = 0; e < ne; ++e) {
        bool ok = d.sigma_t[e] > 0.0;
        for (int f = 0; f < 4 && ok; ++f) {
          const bool in = (mk[e] >> f) & 1u;
          for (int q = 0; q < nq && ok; ++q) {
            const double *g = &o.geo_f[(((size_t)e * 4 + f) * nq + q) * 2];
            const double on = ox * g[0] + oy * g[1];
            ok = in ? on <= 0.0 : on >= 0.0;
          }
        }
        if (!ok) {
          mk[e] |= (uint8_t)0x80;
          ++o.n_pivoting;
        }
      }
    }
  }

  // affine maps: J and adj(F) equal at every volume point to rounding, and
  // n ds along each face equal to the face chord.  The map derivatives are
  // sums of control-point coordinates times O(1) basis derivatives, so their
  // rounding error scales with the size of the coordinates (R), not with the
  // element: on fine meshes far from the origin it is many times 1e-13 of
  // the derivatives themselves.
  o.affine = o.straight;
  for (int e = 0; e < ne && o.affine; ++e) {
    const double *g0 = &o.geo_v[(size_t)e * o.Q * 5];
    const double w0 = T.gw[0] * T.gw[0];
    double scale = 0.0, R = 0.0;
    for (int k = 1; k < 5; ++k) scale = std::max(scale, std::fabs(g0[k] / w0));
    for (int li = 0; li < ncp_e; ++li) {
      const double *x = d.cp_xy + 2 * (size_t)d.elem_cp[(size_t)e * ncp_e + li];
      R = std::max(R, std::max(std::fabs(x[0]), std::fabs(x[1])));
    }
    const double tol_adj = 1e-13 * scale + eps_geo * R;
    const double tol_J = 1e-13 * std::fabs(g0[0] / w0) + 2.0 * scale * eps_geo * R;
    for (int q = 1; q < o.Q && o.affine; ++q) {
      const double *gq = &o.geo_v[((size_t)e * o.Q + q) * 5];
      const double wq = T.gw[q % nq] * T.gw[q / nq];
      if (std::fabs(gq[0] / wq - g0[0] / w0) > tol_J) o.affine = false;
      for (int k = 1; k < 5; ++k)
        if (std::fabs(gq[k] / wq - g0[k] / w0) > tol_adj) o.affine = false;
    }
  }
  if (o.affine) {
    o.geo_a.assign((size_t)ne * 16, 0.0);
    const double w0 = T.gw[0] * T.gw[0];
    for (int e = 0; e < ne; ++e) {
      const double *g0 = &o.geo_v[(size_t)e * o.Q * 5];
      double *ga = &o.geo_a[(size_t)e * 16];
      for (int k = 0; k < 5; ++k) ga[k] = g0[k] / w0;
      for (int f = 0; f < 4; ++f) {
        ga[5 + 2 * f] = chord[8 * e + 2 * f];
        ga[6 + 2 * f] = chord[8 * e + 2 * f + 1];
      }
    }
  }

  o.omega.assign(d.omega, d.omega + 2 * nd);
  o.weight.assign(d.weight, d.weight + nd);
  o.sigma_t.assign(d.sigma_t, d.sigma_t + ne);
  o.sigma_s.assign(d.sigma_s, d.sigma_s + ne);
  return VEF_OK;
}

}  // namespace vefplan

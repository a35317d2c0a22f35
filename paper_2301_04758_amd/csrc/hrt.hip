// Element-local blocks of the hybridized Raviart-Thomas VEF method and their
// inverse (Olivier & Haut, Sec. 7, "Implementation Details": the local
// matrices A_hat, G_hat, D_hat, M_a and the blocks W, X, Y, Z of Eq.
// eq:block_inv), for affine elements.
//
// One wave per element; lane r owns row r of the local block matrix
//   [[A, G], [D, Ma]]   (nv + nphi rows: RT_p current, then Q_p scalar flux).
// On an affine element the contravariant Piola map (Eq. eq:piola) has a
// constant F and J, and its gradient (Eq. eq:piola_grad) has no correction
// term, so every entry is a reference-space sum:
//   A_ij = sum_q w_q sigma_t / J  vh_i . (F^T F) vh_j
//          + boundary faces: sum_q w_q |N_f| / (E_b J^2) (vh_i . F^T E n)(vh_j . F^T n)
//   G_ij = - sum_q w_q (grad vh_i : F^T E F^{-T}) uh_j
//   D_ij = sum_q w_q uh_i div vh_j,   Ma_ij = sum_q w_q sigma_a J uh_i uh_j.
// E = P / phi at each point from the transport moments (isotropic I/3 where
// phi <= 0); E_b as given by the closures (1/2 where not positive).  Only G
// varies from point to point with E; the volume parts of A, D and Ma are
// reference matrices (built on the host) scaled by the element's constants.
//
// The inverse is in-place Gauss-Jordan in natural order: the current
// unknowns (A, symmetric positive definite for sigma_t > 0) are eliminated
// first, then the Schur complement S = Ma - D A^{-1} G -- the block
// elimination behind the formulas for W, X, Y, Z, which assume A and S
// non-singular and allow a singular Ma.  Every lane reads the pivot row from
// the pivot lane's registers (fully unrolled, so every index is a
// compile-time constant).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace vefk {

namespace {

constexpr int kHrtWaves = 4;  // elements (waves) per work-group
// Resident waves per SIMD the register allocation must allow (512 / w
// VGPRs each): the elimination is a chain of lane reads and dependent FMAs
// whose latency the other waves hide; the row of the block matrix
// (2 (p+1)(p+2) + (p+1)^2 doubles per lane) sets how many fit without spills.
constexpr int hrt_waves_per_simd(int p) { return p == 1 ? 4 : p == 2 ? 3 : 2; }

template <int P, int NQ>
struct Hrt {
  static constexpr int NX = (P + 2) * (P + 1);
  static constexpr int NV = 2 * NX;
  static constexpr int NPHI = (P + 1) * (P + 1);
  static constexpr int NT = (P + 1) * (P + 1);
  static constexpr int N = NV + NPHI;
  static constexpr int Q = NQ * NQ;
  static constexpr int OFF_W = 0;
  static constexpr int OFF_VR = OFF_W + Q;
  static constexpr int OFF_DR = OFF_VR + Q * NV;
  static constexpr int OFF_U = OFF_DR + 2 * Q * NV;
  static constexpr int OFF_TV = OFF_U + Q * NPHI;
  static constexpr int OFF_VRF = OFF_TV + Q * NT;
  static constexpr int OFF_TF = OFF_VRF + 4 * NQ * NV;
  static constexpr int OFF_WF = OFF_TF + 4 * NQ * NT;
  static constexpr int OFF_MV = OFF_WF + NQ;
  static constexpr int OFF_DV = OFF_MV + NV * NV;
  static constexpr int OFF_MU = OFF_DV + NPHI * NV;
  static constexpr int OFF_LF = OFF_MU + NPHI * NPHI;
  static constexpr int OFF_LR = OFF_LF + NQ * (P + 1);
  static_assert(N <= 64, "one row per lane");
};

// 1 / d: the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - d r) (each roughly doubles the correct bits).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// The value of x in lane src (uniform), as two 32-bit lane reads.
__device__ __forceinline__ double lane_value(double x, int src) {
  const unsigned long long b = __double_as_longlong(x);
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<unsigned>(b), src);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<unsigned>(b >> 32), src);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// E = P / phi at one point from nodal transport moments (basis values b)
template <int NT>
__device__ __forceinline__ void eddington_at(const double *__restrict__ mom, size_t ne_nt, size_t off,
                                             const double *__restrict__ b, double &exx, double &exy, double &eyy) {
  double ph = 0.0, pxx = 0.0, pxy = 0.0, pyy = 0.0;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    ph += b[j] * mom[off + j];
    pxx += b[j] * mom[3 * ne_nt + off + j];
    pxy += b[j] * mom[4 * ne_nt + off + j];
    pyy += b[j] * mom[5 * ne_nt + off + j];
  }
  if (ph > 0.0) {
    exx = pxx / ph;
    exy = pxy / ph;
    eyy = pyy / ph;
  } else {
    exx = eyy = 1.0 / 3.0;
    exy = 0.0;
  }
}

template <int P, int NQ>
__global__ void __launch_bounds__(64 * kHrtWaves, hrt_waves_per_simd(P))
k_hrt_inverse(const double *__restrict__ tab, const double *__restrict__ geo, const double *__restrict__ sig,
              const int32_t *__restrict__ nbr, const double *__restrict__ mom, const double *__restrict__ Eb,
              int ne, double *__restrict__ out) {
  using H = Hrt<P, NQ>;
  constexpr int NX = H::NX, NV = H::NV, NPHI = H::NPHI, NT = H::NT, N = H::N, Q = H::Q;
  __shared__ double sT[kHrtWaves][Q][4];   // F^T E F^{-T} at volume points
  __shared__ double sF[kHrtWaves][NQ][4];  // E at the points of one boundary face, and 1 / E_b
  constexpr int kTile = (N * N * kHrtWaves * 8 <= 40 * 1024) ? N * N : 1;
  __shared__ __align__(16) double sTile[kHrtWaves][kTile];  // output block of one element
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * kHrtWaves + w;
  if (e >= ne) return;  // whole waves only; the kernel has no work-group barrier

  const double *g = geo + (size_t)e * 13;  // J, adj(F) row major, face chords N_0..N_3
  const double J = g[0];
  const double F00 = g[4], F01 = -g[2], F10 = -g[3], F11 = g[1];
  // F^{-T} = adj(F)^T / J
  const double Fi00 = g[1] / J, Fi01 = g[3] / J, Fi10 = g[2] / J, Fi11 = g[4] / J;
  const double G00 = F00 * F00 + F10 * F10, G01 = F00 * F01 + F10 * F11, G11 = F01 * F01 + F11 * F11;
  const double st = sig[2 * (size_t)e], sa = st - sig[2 * (size_t)e + 1];
  const size_t ne_nt = (size_t)ne * NT, off_e = (size_t)e * NT;

  // E at the volume points, transformed: T = F^T E F^{-T}
  if (lane < Q) {
    double exx, exy, eyy;
    eddington_at<NT>(mom, ne_nt, off_e, tab + H::OFF_TV + lane * NT, exx, exy, eyy);
    // F^T E
    const double a00 = F00 * exx + F10 * exy, a01 = F00 * exy + F10 * eyy;
    const double a10 = F01 * exx + F11 * exy, a11 = F01 * exy + F11 * eyy;
    sT[w][lane][0] = a00 * Fi00 + a01 * Fi10;
    sT[w][lane][1] = a00 * Fi01 + a01 * Fi11;
    sT[w][lane][2] = a10 * Fi00 + a11 * Fi10;
    sT[w][lane][3] = a10 * Fi01 + a11 * Fi11;
  }
  __builtin_amdgcn_wave_barrier();

  const int r = lane;
  const bool cur = r < NV;           // current test function v_r
  const int rc = r < NX ? 0 : 1;     // its non-zero component
  const int rv = cur ? r : 0;        // table index (clamped for other lanes)
  const int rp = (r >= NV && r < N) ? r - NV : 0;
  // Volume terms.  Only G needs the sum over the points (E varies); A, D
  // and Ma are reference matrices scaled by the element's constants:
  //   A_ij = sigma_t / J (F^T F)_{c_i c_j} MV_ij, D = DV, Ma = sigma_a J MU.
  double a[N];
  if (cur) {
    const double *mv = tab + H::OFF_MV + rv * NV;
    const double s0 = st / J * (rc == 0 ? G00 : G01), s1 = st / J * (rc == 0 ? G01 : G11);
#pragma unroll
    for (int j = 0; j < NX; ++j) a[j] = s0 * mv[j];
#pragma unroll
    for (int j = NX; j < NV; ++j) a[j] = s1 * mv[j];
  } else {
    const double *dv = tab + H::OFF_DV + rp * NV;
    const double *mu = tab + H::OFF_MU + rp * NPHI;
#pragma unroll
    for (int j = 0; j < NV; ++j) a[j] = dv[j];
#pragma unroll
    for (int j = 0; j < NPHI; ++j) a[NV + j] = sa * J * mu[j];
  }
  if (cur) {
#pragma unroll
    for (int j = 0; j < NPHI; ++j) a[NV + j] = 0.0;
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
      const double *dr = tab + H::OFF_DR + q * NV * 2;
      const double *u = tab + H::OFF_U + q * NPHI;
      const double dxi = dr[2 * rv], dyi = dr[2 * rv + 1];
      const double gT = rc == 0 ? dxi * sT[w][q][0] + dyi * sT[w][q][1] : dxi * sT[w][q][2] + dyi * sT[w][q][3];
      const double cg = -tab[H::OFF_W + q] * gT;
#pragma unroll
      for (int j = 0; j < NPHI; ++j) a[NV + j] += cg * u[j];
    }
  }

  // boundary faces: (1/E_b) (v . E n)(J . n)
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const int nb = nbr[4 * (size_t)e + f];
    if (nb >= 0) continue;
    const int bf = -nb - 1;
    if (lane < NQ) {
      double exx, exy, eyy;
      eddington_at<NT>(mom, ne_nt, off_e, tab + H::OFF_TF + (f * NQ + lane) * NT, exx, exy, eyy);
      const double eb = Eb ? Eb[(size_t)bf * NQ + lane] : 0.5;
      sF[w][lane][0] = exx;
      sF[w][lane][1] = exy;
      sF[w][lane][2] = eyy;
      sF[w][lane][3] = 1.0 / (eb > 0.0 ? eb : 0.5);
    }
    __builtin_amdgcn_wave_barrier();
    const double cx = g[5 + 2 * f], cy = g[6 + 2 * f];
    const double len = sqrt(cx * cx + cy * cy), nx = cx / len, ny = cy / len;
    const double tn0 = F00 * nx + F10 * ny, tn1 = F01 * nx + F11 * ny;  // t_c . n
    if (cur) {
#pragma unroll 1
      for (int q = 0; q < NQ; ++q) {
        const double *vf = tab + H::OFF_VRF + (f * NQ + q) * NV;
        const double enx = sF[w][q][0] * nx + sF[w][q][1] * ny, eny = sF[w][q][1] * nx + sF[w][q][2] * ny;
        const double ten = rc == 0 ? F00 * enx + F10 * eny : F01 * enx + F11 * eny;  // t_{c_r} . E n
        const double c = tab[H::OFF_WF + q] * len * sF[w][q][3] / (J * J) * vf[rv] * ten;
        const double c0 = c * tn0, c1 = c * tn1;
#pragma unroll
        for (int j = 0; j < NX; ++j) a[j] += c0 * vf[j];
#pragma unroll
        for (int j = NX; j < NV; ++j) a[j] += c1 * vf[j];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }

  // in-place Gauss-Jordan inversion, natural order.  Step k: every lane
  // reads the pivot row from lane k's registers (readlane: no LDS round trip
  // on the dependency chain of the steps) and eliminates entry k from its
  // own row,  a_j <- a_j - g row_j,  g = a_k / a_kk,  a_k <- -g.
  // The pivot row is not divided by a_kk at its step: it keeps its values
  // with a 1 in column k, and its lane remembers 1 / a_kk.  Later steps treat
  // the row linearly, so one multiplication by that factor at the end gives
  // the row of the inverse; this saves a multiply per entry and step.
  double rscale = 1.0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const bool me = lane == k;
    double row[N];
#pragma unroll
    for (int j = 0; j < N; ++j) row[j] = lane_value(a[j], k);
    const double pinv = recip(row[k]);
    const double gk = me ? 0.0 : a[k] * pinv;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != k) a[j] = fma(-gk, row[j], a[j]);
    a[k] = me ? 1.0 : -gk;
    rscale = me ? pinv : rscale;
  }
#pragma unroll
  for (int j = 0; j < N; ++j) a[j] *= rscale;

  double *o = out + (size_t)e * N * N;
  if constexpr (N * N * kHrtWaves * 8 <= 40 * 1024) {
    // through LDS, so that the element's N x N block is written contiguously
    // (each store instruction covers 64 consecutive doubles)
    double *tile = sTile[w];
    if (r < N) {
#pragma unroll
      for (int j = 0; j < N; ++j) tile[r * N + j] = a[j];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < (N * N + 63) / 64; ++t) {
      const int i = lane + 64 * t;
      if (i < N * N) o[i] = tile[i];
    }
  } else if (r < N) {
#pragma unroll
    for (int j = 0; j < N; ++j) o[r * N + j] = a[j];
  }
}

// Element-local part of the hybridized solve (Sec. 7): the couplings of the
// element's current to the multipliers of its interior faces,
//   C1[(f,t)][i] = int_F mu_t (v_i . n) ds,
//   C2[i][(f,t)] = int_F (v_i . <E n>) mu_t ds   (<E n>: E n averaged over
//                                                  the face's two sides),
// the right-hand sides g_i = int v_i . Q1 + boundary faces
// 2 int (1/E_b) (v_i . E n) J_in ds and f_j = int u_j Q0, and from the
// block inverse inv = [[W, X], [Y, Z]]:
//   sol0 = inv [g; f],  resp = inv [C2; 0]      (the element's [J; phi] is
//                                                 sol0 - resp lambda),
//   hloc = C1 resp_J = C1 W C2,  rloc = C1 sol0_J = C1 (W g + X f),
// the element's contributions to H lambda = r.  One wave per element; lane i
// owns test function i for C1, C2, g and f, and row i of the products.
template <int P, int NQ>
__global__ void __launch_bounds__(64 * kHrtWaves)
k_hrt_reduce(const double *__restrict__ tab, const double *__restrict__ geo, const int32_t *__restrict__ nbr,
             const int8_t *__restrict__ nbr_face, const double *__restrict__ mom, const double *__restrict__ Eb,
             const double *__restrict__ Jin, const double *__restrict__ Q0, const double *__restrict__ Q1, int ne,
             const double *__restrict__ inv, double *__restrict__ hloc, double *__restrict__ rloc,
             double *__restrict__ sol0, double *__restrict__ resp) {
  using H = Hrt<P, NQ>;
  constexpr int NX = H::NX, NV = H::NV, NPHI = H::NPHI, NT = H::NT, N = H::N, Q = H::Q, P1 = P + 1;
  constexpr int NL = 4 * P1;  // multiplier slots of the element: (face, node)
  __shared__ double sE[kHrtWaves][2][4][NQ][3];  // E at the face points: own side, other side
  __shared__ double sB[kHrtWaves][N];             // [g; f]
  __shared__ double sC1[kHrtWaves][NL][NV];
  __shared__ double sC2[kHrtWaves][NV][NL];
  __shared__ double sR[kHrtWaves][NV][NL];        // resp rows of the current unknowns
  __shared__ double sS[kHrtWaves][NV];            // sol0 of the current unknowns
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * kHrtWaves + w;
  if (e >= ne) return;  // whole waves only; the kernel has no work-group barrier
  const double *g = geo + (size_t)e * 13;
  const double J = g[0];
  const double F00 = g[4], F01 = -g[2], F10 = -g[3], F11 = g[1];
  const size_t ne_nt = (size_t)ne * NT;

  // E at the face points, this element's side and the neighbour's (the
  // neighbour runs the face the other way: its point NQ-1-q is point q here)
  if (lane < 8 * NQ) {
    const int side = lane / (4 * NQ), f = (lane / NQ) & 3, q = lane % NQ;
    int el = e, ff = f, qq = q;
    const int nb = nbr[4 * (size_t)e + f];
    if (side == 1) {
      if (nb >= 0) {
        el = nb;
        ff = nbr_face[4 * (size_t)e + f];
        qq = NQ - 1 - q;
      }
    }
    double exx, exy, eyy;
    eddington_at<NT>(mom, ne_nt, (size_t)el * NT, tab + H::OFF_TF + (ff * NQ + qq) * NT, exx, exy, eyy);
    sE[w][side][f][q][0] = exx;
    sE[w][side][f][q][1] = exy;
    sE[w][side][f][q][2] = eyy;
  }
  __builtin_amdgcn_wave_barrier();

  const int r = lane;
  const bool cur = r < NV;
  const int rc = r < NX ? 0 : 1;  // non-zero component of v_r
  const int rv = cur ? r : 0;
  // (F^T a)_c / J for the component c of v_r: v_r . a = vhat_r (F^T a)_c / J
  auto ft = [&](double ax, double ay) { return (rc == 0 ? F00 * ax + F10 * ay : F01 * ax + F11 * ay) / J; };
  double bval = 0.0;
  if (cur) {
    // volume: g_r = sum_q w_q vhat_r(q) (F^T Q1_q)_c
    for (int q = 0; q < Q; ++q) {
      const double qx = Q1[(size_t)e * Q + q], qy = Q1[((size_t)ne + e) * Q + q];
      bval += tab[H::OFF_W + q] * tab[H::OFF_VR + q * NV + rv] * (rc == 0 ? F00 * qx + F10 * qy : F01 * qx + F11 * qy);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double cx = g[5 + 2 * f], cy = g[6 + 2 * f];
      const double len = sqrt(cx * cx + cy * cy), nx = cx / len, ny = cy / len;
      const int nb = nbr[4 * (size_t)e + f];
      double c1[P1], c2[P1];
#pragma unroll
      for (int t = 0; t < P1; ++t) c1[t] = c2[t] = 0.0;
      if (nb >= 0) {
        const double *lam = tab + (e < nb ? H::OFF_LF : H::OFF_LR);
        const double vn = ft(nx, ny);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double wv = tab[H::OFF_WF + q] * len * tab[H::OFF_VRF + (f * NQ + q) * NV + rv];
          const double *a = sE[w][0][f][q], *b = sE[w][1][f][q];
          const double exx = 0.5 * (a[0] + b[0]), exy = 0.5 * (a[1] + b[1]), eyy = 0.5 * (a[2] + b[2]);
          const double ven = ft(exx * nx + exy * ny, exy * nx + eyy * ny);
#pragma unroll
          for (int t = 0; t < P1; ++t) {
            c1[t] += wv * lam[q * P1 + t] * vn;
            c2[t] += wv * lam[q * P1 + t] * ven;
          }
        }
      } else {
        const int bf = -nb - 1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double eb0 = Eb ? Eb[(size_t)bf * NQ + q] : 0.5;
          const double eb = eb0 > 0.0 ? eb0 : 0.5;
          const double *a = sE[w][0][f][q];
          const double ven = ft(a[0] * nx + a[1] * ny, a[1] * nx + a[2] * ny);
          bval += 2.0 * tab[H::OFF_WF + q] * len / eb * tab[H::OFF_VRF + (f * NQ + q) * NV + rv] * ven *
                  Jin[(size_t)bf * NQ + q];
        }
      }
#pragma unroll
      for (int t = 0; t < P1; ++t) {
        sC1[w][f * P1 + t][rv] = c1[t];
        sC2[w][rv][f * P1 + t] = c2[t];
      }
    }
  } else if (r < N) {
    // f_j = sum_q w_q J Q0_q u_j(q)
    const int j = r - NV;
    for (int q = 0; q < Q; ++q) bval += tab[H::OFF_W + q] * J * Q0[(size_t)e * Q + q] * tab[H::OFF_U + q * NPHI + j];
  }
  if (r < N) sB[w][r] = bval;
  __builtin_amdgcn_wave_barrier();

  // row r of sol0 = inv [g; f] and of resp = inv [C2; 0]
  if (r < N) {
    const double *ir = inv + ((size_t)e * N + r) * N;
    double s0 = 0.0, rr[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) rr[a] = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const double x = ir[j];
      s0 += x * sB[w][j];
      if (j < NV) {
#pragma unroll
        for (int a = 0; a < NL; ++a) rr[a] += x * sC2[w][j][a];
      }
    }
    sol0[(size_t)e * N + r] = s0;
#pragma unroll
    for (int a = 0; a < NL; ++a) resp[((size_t)e * N + r) * NL + a] = rr[a];
    if (r < NV) {
      sS[w][r] = s0;
#pragma unroll
      for (int a = 0; a < NL; ++a) sR[w][r][a] = rr[a];
    }
  }
  __builtin_amdgcn_wave_barrier();

  // hloc = C1 resp_J, rloc = C1 sol0_J
  for (int idx = lane; idx < NL * NL + NL; idx += 64) {
    const int a = idx < NL * NL ? idx / NL : idx - NL * NL;
    const int b = idx < NL * NL ? idx % NL : -1;
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) acc += sC1[w][a][i] * (b >= 0 ? sR[w][i][b] : sS[w][i]);
    if (b >= 0)
      hloc[((size_t)e * NL + a) * NL + b] = acc;
    else
      rloc[(size_t)e * NL + a] = acc;
  }
}

template <int P, int NQ>
hipError_t launch_reduce_t(const HrtReduceLaunch &L) {
  const int grid = (L.ne + kHrtWaves - 1) / kHrtWaves;
  hipLaunchKernelGGL((k_hrt_reduce<P, NQ>), dim3(grid), dim3(64 * kHrtWaves), 0, L.stream, L.tab, L.geo, L.nbr,
                     L.nbr_face, L.mom, L.Eb, L.Jin, L.Q0, L.Q1, L.ne, L.inv, L.hloc, L.rloc, L.sol0, L.resp);
  return hipGetLastError();
}

template <int P, int NQ>
hipError_t launch_hrt_t(const HrtLaunch &L) {
  const int grid = (L.ne + kHrtWaves - 1) / kHrtWaves;
  hipLaunchKernelGGL((k_hrt_inverse<P, NQ>), dim3(grid), dim3(64 * kHrtWaves), 0, L.stream, L.tab, L.geo, L.sig, L.nbr,
                     L.mom, L.Eb, L.ne, L.out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_hrt_reduce(const HrtReduceLaunch &L) {
  if (L.ne <= 0) return hipSuccess;
  switch (L.p * 16 + L.nq) {
    case 1 * 16 + 3: return launch_reduce_t<1, 3>(L);
    case 1 * 16 + 4: return launch_reduce_t<1, 4>(L);
    case 2 * 16 + 4: return launch_reduce_t<2, 4>(L);
    case 2 * 16 + 5: return launch_reduce_t<2, 5>(L);
    case 3 * 16 + 5: return launch_reduce_t<3, 5>(L);
    case 3 * 16 + 6: return launch_reduce_t<3, 6>(L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hrt_inverse(const HrtLaunch &L) {
  if (L.ne <= 0) return hipSuccess;
  switch (L.p * 16 + L.nq) {
    case 1 * 16 + 3: return launch_hrt_t<1, 3>(L);
    case 1 * 16 + 4: return launch_hrt_t<1, 4>(L);
    case 2 * 16 + 4: return launch_hrt_t<2, 4>(L);
    case 2 * 16 + 5: return launch_hrt_t<2, 5>(L);
    case 3 * 16 + 5: return launch_hrt_t<3, 5>(L);
    case 3 * 16 + 6: return launch_hrt_t<3, 6>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vefk

// HIP kernels for gfx950: level-synchronous DG S_N sweep, angular-moment and
// residual reduction, boundary sums and VEF closures.
//
// Sweep work mapping (one launch per upwind level): a "slot" of SLOT lanes
// (the power of two >= n = (p+1)^2) of one 64-wide wavefront owns one
// element-direction solve; lane r owns row r (test function r) of the local
// system.  Each lane assembles its row by quadrature from the per-element
// geometry factors (w J and w adj(F) at volume points, w n ds at face points)
// and the basis tables staged in LDS; inflow traces come from the upwind
// element's face nodes (Gauss-Lobatto nodes include the element boundary, so
// a face trace is the p+1 face-node values, read in reversed order because
// the two sides run the shared face in opposite senses).  The system is solved
// by Gauss-Jordan elimination with partial pivoting across the slot's lanes
// (pivot search and pivot-row broadcast by cross-lane shuffles), so each lane
// ends with one unknown.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace vefk {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

template <int P>
struct Shape {
  static constexpr int P1 = P + 1;
  static constexpr int N = P1 * P1;
  static constexpr int SLOT = N <= 4 ? 4 : (N <= 8 ? 8 : (N <= 16 ? 16 : 32));
  static constexpr int SPW = 64 / SLOT;
};

// node index of position c (counter-clockwise) along face f
template <int P>
__device__ __forceinline__ int face_node(int f, int c) {
  constexpr int P1 = P + 1;
  switch (f) {
    case 0: return c;
    case 1: return P + P1 * c;
    case 2: return (P - c) + P1 * P;
    default: return P1 * (P - c);
  }
}

template <typename T>
__device__ __forceinline__ T ld(const double *p, size_t i) {
  return static_cast<T>(p[i]);
}

template <int P, int NQ, typename T>
__global__ void __launch_bounds__(256)
k_sweep_level(const int2 *__restrict__ solves, int n_solves, const KProb *__restrict__ probs,
              const KIO *__restrict__ io, const T *__restrict__ tables, int it,
              const int *__restrict__ stop, int *__restrict__ status) {
  using S = Shape<P>;
  constexpr int P1 = S::P1, N = S::N, SLOT = S::SLOT, SPW = S::SPW;
  constexpr int Q = NQ * NQ;
  __shared__ T sV[Q * N];
  __shared__ T sDx[Q * N];
  __shared__ T sDy[Q * N];
  __shared__ T sF[NQ * P1];
  if (*stop) return;
  for (int i = threadIdx.x; i < Q * N; i += blockDim.x) {
    sV[i] = tables[i];
    sDx[i] = tables[Q * N + i];
    sDy[i] = tables[2 * Q * N + i];
  }
  for (int i = threadIdx.x; i < NQ * P1; i += blockDim.x) sF[i] = tables[3 * Q * N + i];
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int r = lane & (SLOT - 1);
  const int sid = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPW + lane / SLOT;
  const bool valid = sid < n_solves;
  const bool row_ok = valid && r < N;
  const int rr = r < N ? r : N - 1;  // table index for padding lanes
  const int a = rr % P1, b = rr / P1;

  int e = 0, d = 0, prob = 0;
  if (valid) {
    const int2 sv = solves[sid];
    e = sv.x;
    d = sv.y & 0xffff;
    prob = sv.y >> 16;
  }
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int ne = pb.ne;
  const T ox = static_cast<T>(pb.omega[2 * d]);
  const T oy = static_cast<T>(pb.omega[2 * d + 1]);
  const T st = static_cast<T>(pb.sig[2 * e]);
  const T ss = static_cast<T>(pb.sig[2 * e + 1] * kInv4Pi);
  const unsigned mask = pb.mask[(size_t)d * ne + e];
  const double *phi = it == 0 ? pio.phi_in : pio.mom;

  // nodal coefficients of the isotropic part of the source
  T s[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T v = T(0);
    if (phi) v = ss * ld<T>(phi, (size_t)e * N + j);
    if (pio.q_iso) v += ld<T>(pio.q_iso, (size_t)e * N + j);
    s[j] = v;
  }

  T A[N];
#pragma unroll
  for (int j = 0; j < N; ++j) A[j] = T(0);
  T rhs = T(0);

  // ---- volume terms
  const T *gv = static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5;
  const double *qd = pio.q_dir ? pio.q_dir + ((size_t)d * ne + e) * Q : nullptr;
#pragma unroll 1
  for (int q = 0; q < Q; ++q) {
    const T wJ = gv[5 * q], a00 = gv[5 * q + 1], a01 = gv[5 * q + 2], a10 = gv[5 * q + 3],
            a11 = gv[5 * q + 4];
    const T gx = a00 * ox + a01 * oy;
    const T gy = a10 * ox + a11 * oy;
    const T li = sV[q * N + rr];
    const T c = st * wJ * li - (gx * sDx[q * N + rr] + gy * sDy[q * N + rr]);
    T src = qd ? static_cast<T>(qd[q]) : T(0);
#pragma unroll
    for (int j = 0; j < N; ++j) src += s[j] * sV[q * N + j];
    rhs += wJ * li * src;
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] += c * sV[q * N + j];
  }

  // ---- face terms
  const T *psi = static_cast<const T *>(pio.psi);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
    const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
    const T *gf = static_cast<const T *>(pb.geo_f) + ((size_t)e * 4 + f) * NQ * 2;
    if (!((mask >> f) & 1u)) {
      if (on_face && row_ok) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
          const T t = on * sF[q * P1 + pos];
#pragma unroll
          for (int c = 0; c < P1; ++c) A[face_node<P>(f, c)] += t * sF[q * P1 + c];
        }
      }
    } else if (on_face && row_ok) {
      const int nb = pb.nbr[4 * e + f];
      if (nb >= 0) {
        const int f2 = pb.nbr_face[4 * e + f];
        const T *up = psi + ((size_t)d * ne + nb) * N;
        T tr[P1];
#pragma unroll
        for (int c = 0; c < P1; ++c) tr[c] = up[face_node<P>(f2, P - c)];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          T ph = T(0);
#pragma unroll
          for (int c = 0; c < P1; ++c) ph += tr[c] * sF[q * P1 + c];
          const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
          rhs -= on * sF[q * P1 + pos] * ph;
        }
      } else if (pio.psi_bc) {
        const double *bc = pio.psi_bc + ((size_t)d * pb.nbf + (-nb - 1)) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
          rhs -= on * sF[q * P1 + pos] * static_cast<T>(bc[q]);
        }
      }
    }
  }

  // ---- Gauss-Jordan elimination with partial pivoting across the slot
  bool active = row_ok;
  int my_k = 0;
  T piv = T(1);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    T v = active ? fabs(A[k]) : T(-1);
    int idx = r;
#pragma unroll
    for (int off = SLOT / 2; off >= 1; off >>= 1) {
      const T ov = __shfl_xor(v, off, SLOT);
      const int oi = __shfl_xor(idx, off, SLOT);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const T pk = __shfl(A[k], idx, SLOT);
    const T pr = __shfl(rhs, idx, SLOT);
    if (r == idx) {
      active = false;
      my_k = k;
      piv = A[k];
      bad = row_ok && !(piv != T(0));
    }
    const T l = (row_ok && r != idx) ? A[k] / pk : T(0);
#pragma unroll
    for (int j = k + 1; j < N; ++j) {
      const T pj = __shfl(A[j], idx, SLOT);
      A[j] -= l * pj;
    }
    rhs -= l * pr;
  }
  if (row_ok) {
    T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
    out[my_k] = rhs / piv;
    if (bad) atomicOr(status, 1);
  }
}

// Angular moments (fixed direction order, double accumulation) and the
// max-norm change of the scalar flux; one thread per (element, node).
template <typename T>
__global__ void __launch_bounds__(256)
k_moments(const KProb *__restrict__ probs, const KIO *__restrict__ io, int prob, int ne_n, int it,
          const int *__restrict__ stop) {
  if (*stop) return;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double diff = 0.0;
  if (i < ne_n) {
    const T *psi = static_cast<const T *>(pio.psi);
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0;
    for (int d = 0; d < pb.nd; ++d) {
      const double v = static_cast<double>(psi[(size_t)d * ne_n + i]);
      const double w = pb.weight[d], ox = pb.omega[2 * d], oy = pb.omega[2 * d + 1];
      const double wv = w * v;
      m0 += wv;
      m1 += wv * ox;
      m2 += wv * oy;
      m3 += wv * ox * ox;
      m4 += wv * ox * oy;
      m5 += wv * oy * oy;
    }
    const double *phi = it == 0 ? pio.phi_in : pio.mom;
    const double old = phi ? phi[i] : 0.0;
    double *mom = pio.mom;
    mom[i] = m0;
    mom[(size_t)ne_n + i] = m1;
    mom[2 * (size_t)ne_n + i] = m2;
    mom[3 * (size_t)ne_n + i] = m3;
    mom[4 * (size_t)ne_n + i] = m4;
    mom[5 * (size_t)ne_n + i] = m5;
    diff = fabs(m0 - old);
  }
  // block max, then one atomic max on the bit pattern (non-negative doubles
  // order like unsigned integers)
  for (int off = 32; off >= 1; off >>= 1) diff = fmax(diff, __shfl_xor(diff, off, 64));
  __shared__ double wmax[16];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = diff;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, wmax[w]);
    if (pio.resid)
      atomicMax(reinterpret_cast<unsigned long long *>(pio.resid + it),
                static_cast<unsigned long long>(__double_as_longlong(mx)));
  }
}

// Boundary sums sum_d w |Omega.n| psi_d and sum_d w psi_d at boundary face
// points (interior trace), one thread per (boundary face, point).
template <typename T>
__global__ void __launch_bounds__(256)
k_boundary(const KProb *__restrict__ probs, const KIO *__restrict__ io, int prob, int nbf, int nq,
           int p, const int *__restrict__ stop) {
  if (*stop) return;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbf * nq) return;
  const int bf = i / nq, q = i % nq;
  const int e = pb.bf_ef[bf] >> 2, f = pb.bf_ef[bf] & 3;
  const int P1 = p + 1, n = P1 * P1;
  const double *g = pb.geo_fd + (((size_t)e * 4 + f) * nq + q) * 2;
  const double len = sqrt(g[0] * g[0] + g[1] * g[1]);
  const double nx = g[0] / len, ny = g[1] / len;
  const double *F = pb.tab_d + 3 * (size_t)pb.Q * n + (size_t)q * P1;
  int nodes[5];
  for (int c = 0; c < P1; ++c) {
    switch (f) {
      case 0: nodes[c] = c; break;
      case 1: nodes[c] = p + P1 * c; break;
      case 2: nodes[c] = (p - c) + P1 * p; break;
      default: nodes[c] = P1 * (p - c); break;
    }
  }
  const T *psi = static_cast<const T *>(pio.psi);
  double num = 0.0, den = 0.0;
  for (int d = 0; d < pb.nd; ++d) {
    const T *u = psi + ((size_t)d * pb.ne + e) * n;
    double tr = 0.0;
    for (int c = 0; c < P1; ++c) tr += static_cast<double>(u[nodes[c]]) * F[c];
    const double w = pb.weight[d];
    num += w * fabs(pb.omega[2 * d] * nx + pb.omega[2 * d + 1] * ny) * tr;
    den += w * tr;
  }
  pb.bnd[2 * (size_t)i] = num;
  pb.bnd[2 * (size_t)i + 1] = den;
}

__global__ void k_run_init(const KIO *__restrict__ io, int n_probs, int n_iter, int *stop,
                           int *iters) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *stop = 0;
    *iters = 0;
  }
  if (i < n_probs * n_iter) {
    double *r = io[i / n_iter].resid;
    if (r) r[i % n_iter] = 0.0;
  }
}

__global__ void k_finalize(const KIO *__restrict__ io, int n_probs, int it, double tol, int *stop,
                           int *iters, int *iters_user) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (*stop) return;
  *iters = it + 1;
  if (iters_user) *iters_user = it + 1;
  if (tol > 0.0) {
    double mx = 0.0;
    for (int k = 0; k < n_probs; ++k)
      if (io[k].resid) mx = fmax(mx, io[k].resid[it]);
    if (mx < tol) *stop = 1;
  }
}

// Closures at volume points (E, Q0, Q1) and boundary points (E_b, J_in).
__global__ void __launch_bounds__(256)
k_closures(const KProb *__restrict__ probs, const KMomIO *__restrict__ mio, int prob, int ne, int Q,
           int nbf, int nq) {
  const KProb &pb = probs[prob];
  const KMomIO &io = mio[prob];
  const int n = pb.n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nvol = ne * Q;
  int bad = 0;
  if (i < nvol) {
    const int e = i / Q, q = i % Q;
    const double *V = pb.tab_d + (size_t)q * n;
    if (io.E && io.mom) {
      const size_t N = (size_t)ne * n;
      double ph = 0, pxx = 0, pxy = 0, pyy = 0;
      for (int j = 0; j < n; ++j) {
        const double v = V[j];
        ph += io.mom[(size_t)e * n + j] * v;
        pxx += io.mom[3 * N + (size_t)e * n + j] * v;
        pxy += io.mom[4 * N + (size_t)e * n + j] * v;
        pyy += io.mom[5 * N + (size_t)e * n + j] * v;
      }
      if (ph > 0.0) {
        io.E[i] = pxx / ph;
        io.E[(size_t)nvol + i] = pxy / ph;
        io.E[2 * (size_t)nvol + i] = pyy / ph;
      } else {
        io.E[i] = io.E[(size_t)nvol + i] = io.E[2 * (size_t)nvol + i] = 0.0;
        bad = 1;
      }
    }
    if (io.Q0 || io.Q1) {
      double qi = 0.0;
      if (io.q_iso)
        for (int j = 0; j < n; ++j) qi += io.q_iso[(size_t)e * n + j] * V[j];
      double s0 = 0, s1 = 0, s2 = 0;
      for (int d = 0; d < pb.nd; ++d) {
        const double qq = qi + (io.q_dir ? io.q_dir[((size_t)d * ne + e) * Q + q] : 0.0);
        const double w = pb.weight[d];
        s0 += w * qq;
        s1 += w * pb.omega[2 * d] * qq;
        s2 += w * pb.omega[2 * d + 1] * qq;
      }
      if (io.Q0) io.Q0[i] = s0;
      if (io.Q1) {
        io.Q1[i] = s1;
        io.Q1[(size_t)nvol + i] = s2;
      }
    }
  } else if (i < nvol + nbf * nq) {
    const int j = i - nvol;
    const int bf = j / nq, q = j % nq;
    if (io.Eb) {
      const double num = pb.bnd[2 * (size_t)j], den = pb.bnd[2 * (size_t)j + 1];
      if (den > 0.0) {
        io.Eb[j] = num / den;
      } else {
        io.Eb[j] = 0.0;
        bad = 1;
      }
    }
    if (io.Jin) {
      const int e = pb.bf_ef[bf] >> 2, f = pb.bf_ef[bf] & 3;
      const double *g = pb.geo_fd + (((size_t)e * 4 + f) * nq + q) * 2;
      const double len = sqrt(g[0] * g[0] + g[1] * g[1]);
      const double nx = g[0] / len, ny = g[1] / len;
      double s = 0.0;
      if (io.psi_bc)
        for (int d = 0; d < pb.nd; ++d) {
          const double on = pb.omega[2 * d] * nx + pb.omega[2 * d + 1] * ny;
          if (on < 0.0) s += pb.weight[d] * on * io.psi_bc[((size_t)d * nbf + bf) * nq + q];
        }
      io.Jin[j] = s;
    }
  }
  if (io.n_nonpos) {
    // count per wavefront, one atomic per wave
    const unsigned long long ballot = __ballot(bad);
    if ((threadIdx.x & 63) == 0 && ballot) atomicAdd(io.n_nonpos, (int)__popcll(ballot));
  }
}

__global__ void k_zero_nonpos(const KMomIO *__restrict__ io, int n_probs) {
  const int i = threadIdx.x;
  if (i < n_probs && io[i].n_nonpos) *io[i].n_nonpos = 0;
}

template <int P, int NQ>
hipError_t launch_variant(bool fp32, const int2 *solves, int n_solves, const KProb *probs,
                          const KIO *io, const void *tables, int it, const int *stop, int *status,
                          int block, hipStream_t s) {
  const int spw = Shape<P>::SPW;
  const int per_block = (block / 64) * spw;
  const int grid = (n_solves + per_block - 1) / per_block;
  if (grid == 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL((k_sweep_level<P, NQ, float>), dim3(grid), dim3(block), 0, s, solves,
                       n_solves, probs, io, static_cast<const float *>(tables), it, stop, status);
  else
    hipLaunchKernelGGL((k_sweep_level<P, NQ, double>), dim3(grid), dim3(block), 0, s, solves,
                       n_solves, probs, io, static_cast<const double *>(tables), it, stop, status);
  return hipGetLastError();
}

template <int P>
hipError_t launch_p(int nq, bool fp32, const int2 *solves, int n_solves, const KProb *probs,
                    const KIO *io, const void *tables, int it, const int *stop, int *status,
                    int block, hipStream_t s) {
  switch (nq - P) {
    case 1: return launch_variant<P, P + 1>(fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 2: return launch_variant<P, P + 2>(fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 3: return launch_variant<P, P + 3>(fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 4: return launch_variant<P, P + 4>(fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_sweep_level(int p, int nq, bool fp32, const int2 *solves, int n_solves,
                              const KProb *probs, const KIO *io, const void *tables, int it,
                              const int *stop, int *status, int block, hipStream_t s) {
  switch (p) {
    case 1: return launch_p<1>(nq, fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 2: return launch_p<2>(nq, fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 3: return launch_p<3>(nq, fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    case 4: return launch_p<4>(nq, fp32, solves, n_solves, probs, io, tables, it, stop, status, block, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_moments(bool fp32, const KProb *probs, const KIO *io, int prob, int ne_n, int it,
                          const int *stop, hipStream_t s) {
  const int grid = (ne_n + 255) / 256;
  if (fp32)
    hipLaunchKernelGGL(k_moments<float>, dim3(grid), dim3(256), 0, s, probs, io, prob, ne_n, it, stop);
  else
    hipLaunchKernelGGL(k_moments<double>, dim3(grid), dim3(256), 0, s, probs, io, prob, ne_n, it, stop);
  return hipGetLastError();
}

hipError_t launch_boundary(bool fp32, const KProb *probs, const KIO *io, int prob, int nbf, int nq,
                           int p, const int *stop, hipStream_t s) {
  const int tot = nbf * nq;
  if (tot == 0) return hipSuccess;
  const int grid = (tot + 255) / 256;
  if (fp32)
    hipLaunchKernelGGL(k_boundary<float>, dim3(grid), dim3(256), 0, s, probs, io, prob, nbf, nq, p, stop);
  else
    hipLaunchKernelGGL(k_boundary<double>, dim3(grid), dim3(256), 0, s, probs, io, prob, nbf, nq, p, stop);
  return hipGetLastError();
}

hipError_t launch_run_init(const KIO *io, int n_probs, int n_iter, int *stop, int *iters,
                           hipStream_t s) {
  const int tot = n_probs * n_iter;
  const int grid = (tot + 255) / 256 > 0 ? (tot + 255) / 256 : 1;
  hipLaunchKernelGGL(k_run_init, dim3(grid), dim3(256), 0, s, io, n_probs, n_iter, stop, iters);
  return hipGetLastError();
}

hipError_t launch_finalize(const KIO *io, int n_probs, int it, double tol, int *stop, int *iters,
                           int *iters_user, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, io, n_probs, it, tol, stop, iters, iters_user);
  return hipGetLastError();
}

hipError_t launch_closures(const KProb *probs, const KMomIO *io, int prob, int ne, int Q, int nbf,
                           int nq, hipStream_t s) {
  const int tot = ne * Q + nbf * nq;
  const int grid = (tot + 255) / 256;
  hipLaunchKernelGGL(k_closures, dim3(grid), dim3(256), 0, s, probs, io, prob, ne, Q, nbf, nq);
  return hipGetLastError();
}

hipError_t launch_zero_nonpos(const KMomIO *io, int n_probs, hipStream_t s) {
  // one thread per problem; n_probs is bounded by the handle (<= 1024)
  hipLaunchKernelGGL(k_zero_nonpos, dim3(1), dim3(1024), 0, s, io, n_probs);
  return hipGetLastError();
}

}  // namespace vefk

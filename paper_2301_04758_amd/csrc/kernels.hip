// HIP kernels for gfx950 besides the sweep itself: angular moments and the
// source-iteration residual, boundary sums, run bookkeeping and the VEF
// closures; plus the dispatch of the sweep launches to the per-degree
// translation units (sweep_p*.hip, device code in sweep_device.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace vefk {

namespace {

// Angular moments (double accumulation) and the max-norm change of the
// scalar flux.  A work-group of 4 waves covers 64 (element, node) entries.
// The direction weights and cosines are staged in LDS first (the handle
// allows at most 1024 directions).  Wave w sums the directions of its
// quarter of the direction list in order, with loads unrolled so several are
// in flight, and wave 0 adds the four partial sums in quarter order, so the
// result does not depend on timing.
constexpr int kMomWaves = 4;
constexpr int kMaxMomDirs = 1024;

template <typename T>
__global__ void __launch_bounds__(64 * kMomWaves)
k_moments(const KProb *__restrict__ probs, const KIO *__restrict__ io, int prob, int ne_n, int it,
          const int *__restrict__ stop) {
  if (*stop) return;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int nd = pb.nd;
  // (w, ox, oy) of the directions, nd entries (the launch sizes the
  // work-group's dynamic LDS to them, which leaves room for more resident
  // work-groups than a table for the most directions would)
  extern __shared__ double3 dirs[];
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    const double wt = pb.weight[d];
    dirs[d] = make_double3(wt, pb.omega[2 * d], pb.omega[2 * d + 1]);
  }
  __syncthreads();
  const int d0 = (nd * w) / kMomWaves, d1 = (nd * (w + 1)) / kMomWaves;
  double m[6] = {0, 0, 0, 0, 0, 0};
  if (i < ne_n) {
    const T *psi = static_cast<const T *>(pio.psi) + i;
#pragma unroll 8
    for (int d = d0; d < d1; ++d) {
      const double v = static_cast<double>(psi[(size_t)d * ne_n]);
      const double3 c = dirs[d];
      const double wv = c.x * v, ox = c.y, oy = c.z;
      m[0] += wv;
      m[1] += wv * ox;
      m[2] += wv * oy;
      m[3] += wv * ox * ox;
      m[4] += wv * ox * oy;
      m[5] += wv * oy * oy;
    }
  }
  __shared__ double part[kMomWaves - 1][6][64];
  if (w > 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) part[w - 1][k][lane] = m[k];
  __syncthreads();
  if (w != 0) return;
  double diff = 0.0;
  if (i < ne_n) {
#pragma unroll
    for (int q = 0; q < kMomWaves - 1; ++q)
#pragma unroll
      for (int k = 0; k < 6; ++k) m[k] += part[q][k][lane];
    const double *phi = it == 0 ? pio.phi_in : pio.mom;
    const double old = phi ? phi[i] : 0.0;
    double *mom = pio.mom;
#pragma unroll
    for (int k = 0; k < 6; ++k) mom[(size_t)k * ne_n + i] = m[k];
    diff = fabs(m[0] - old);
  }
  // wave max, then one atomic max on the bit pattern (non-negative doubles
  // order like unsigned integers)
  for (int off = 32; off >= 1; off >>= 1) diff = fmax(diff, __shfl_xor(diff, off, 64));
  if (lane == 0 && pio.resid)
    atomicMax(reinterpret_cast<unsigned long long *>(pio.resid + it),
              static_cast<unsigned long long>(__double_as_longlong(diff)));
}

// Boundary sums sum_d w |Omega.n| psi_d and sum_d w psi_d at boundary face
// points (interior trace).  One wave per boundary face: lane l takes the
// directions l, l + 64, ..., reads the face's nodal values of psi once per
// direction and evaluates the trace at every point of the face; a butterfly
// over the lanes in a fixed order then completes each point's sums.
constexpr int kBndMaxNq = 8;
template <typename T>
__global__ void __launch_bounds__(256)
k_boundary(const KProb *__restrict__ probs, const KIO *__restrict__ io, int prob, int nbf, int nq,
           int p, const int *__restrict__ stop) {
  if (stop && *stop) return;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int bf = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (bf >= nbf) return;  // whole waves
  const int e = pb.bf_ef[bf] >> 2, f = pb.bf_ef[bf] & 3;
  const int P1 = p + 1, n = P1 * P1;
  const double *F = pb.tab_d + 3 * (size_t)pb.Q * n;  // 1D basis at the face points [nq][p+1]
  int nodes[5];
  for (int c = 0; c < P1; ++c) {
    switch (f) {
      case 0: nodes[c] = c; break;
      case 1: nodes[c] = p + P1 * c; break;
      case 2: nodes[c] = (p - c) + P1 * p; break;
      default: nodes[c] = P1 * (p - c); break;
    }
  }
  double nx[kBndMaxNq], ny[kBndMaxNq], num[kBndMaxNq], den[kBndMaxNq];
#pragma unroll
  for (int q = 0; q < kBndMaxNq; ++q) {
    nx[q] = ny[q] = num[q] = den[q] = 0.0;
    if (q < nq) {
      const double *g = pb.geo_fd + (((size_t)e * 4 + f) * nq + q) * 2;
      const double len = sqrt(g[0] * g[0] + g[1] * g[1]);
      nx[q] = g[0] / len;
      ny[q] = g[1] / len;
    }
  }
  const T *psi = static_cast<const T *>(pio.psi);
  for (int d = lane; d < pb.nd; d += 64) {
    const T *u = psi + ((size_t)d * pb.ne + e) * n;
    double uc[5];
    for (int c = 0; c < P1; ++c) uc[c] = static_cast<double>(u[nodes[c]]);
    const double w = pb.weight[d], ox = pb.omega[2 * d], oy = pb.omega[2 * d + 1];
#pragma unroll
    for (int q = 0; q < kBndMaxNq; ++q) {
      if (q >= nq) continue;
      double tr = 0.0;
      for (int c = 0; c < P1; ++c) tr += uc[c] * F[q * P1 + c];
      num[q] += w * fabs(ox * nx[q] + oy * ny[q]) * tr;
      den[q] += w * tr;
    }
  }
#pragma unroll
  for (int q = 0; q < kBndMaxNq; ++q) {
    if (q >= nq) continue;
    double a = num[q], b = den[q];
    for (int off = 32; off >= 1; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    if (lane == q) {
      pb.bnd[2 * ((size_t)bf * nq + q)] = a;
      pb.bnd[2 * ((size_t)bf * nq + q) + 1] = b;
    }
  }
}

__global__ void k_run_init(const KIO *__restrict__ io, int n_probs, int n_iter, int *stop,
                           int *iters, int *status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *stop = 0;
    *iters = 0;
    *status = 0;  // the status word reports the current run only
  }
  if (i < n_probs * n_iter) {
    double *r = io[i / n_iter].resid;
    if (r) r[i % n_iter] = 0.0;
  }
}

__global__ void k_zero_ints(int *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
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
// The direction weights and cosines are staged in LDS as (w, w ox, w oy);
// without a direction-dependent source, Q0 and Q1 at a point are q_iso times
// the sums of those over the directions, formed once per work-group in
// direction order (so every work-group has the same values).  A work-group
// takes chunks of 256 points in turn, so this setup is paid once per
// work-group.  STAGE: the basis table V [Q][n] and, per chunk, its elements'
// phi, Pxx, Pxy, Pyy and q_iso coefficients go through LDS first, read with
// consecutive addresses (the host checks that they fit: kClStageEl elements'
// worth, kClStageV table entries).
constexpr int kClThreads = 256;
constexpr int kClStageEl = 320;   // element-node entries per staged array
constexpr int kClStageV = 49 * 25;
constexpr int kClMaxGroups = 2048;
template <bool STAGE>
__global__ void __launch_bounds__(kClThreads)
k_closures(const KProb *__restrict__ probs, const KMomIO *__restrict__ mio, int prob, int ne, int Q,
           int nbf, int nq) {
  __shared__ double3 dirs[kMaxMomDirs];
  __shared__ double wsum[3];
  __shared__ double sV[STAGE ? kClStageV : 1];
  __shared__ double sM[STAGE ? 5 : 1][STAGE ? kClStageEl : 1];  // phi, Pxx, Pxy, Pyy, q_iso
  const KProb &pb = probs[prob];
  const KMomIO &io = mio[prob];
  const int n = pb.n;
  const int nd = pb.nd;
  for (int d = threadIdx.x; d < nd; d += blockDim.x) {
    const double w = pb.weight[d];
    dirs[d] = make_double3(w, w * pb.omega[2 * d], w * pb.omega[2 * d + 1]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int d = 0; d < nd; ++d) {
      s0 += dirs[d].x;
      s1 += dirs[d].y;
      s2 += dirs[d].z;
    }
    wsum[0] = s0;
    wsum[1] = s1;
    wsum[2] = s2;
  }
  const int nvol = ne * Q;
  const int total = nvol + nbf * nq;
  const size_t N = (size_t)ne * n;
  if constexpr (STAGE)
    for (int x = threadIdx.x; x < Q * n; x += blockDim.x) sV[x] = pb.tab_d[x];
  // chunks of blockDim points, the work-group's every gridDim-th: the
  // direction sums and the basis table above are staged once per work-group
  for (int i0 = blockIdx.x * blockDim.x; i0 < total; i0 += gridDim.x * blockDim.x) {
    const int i = i0 + threadIdx.x;
    // the chunk's elements (volume points i0 .. i0 + 255)
    const int e0 = i0 < nvol ? i0 / Q : 0;
    const int e1 = i0 < nvol ? ((i0 + (int)blockDim.x < nvol ? i0 + (int)blockDim.x : nvol) - 1) / Q + 1 : 0;
    if constexpr (STAGE) {
      __syncthreads();  // the previous chunk's reads of sM are done
      const int cnt = (e1 - e0) * n;
      const size_t b0 = (size_t)e0 * n;
      for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
        if (io.mom) {
          sM[0][x] = io.mom[b0 + x];
          sM[1][x] = io.mom[3 * N + b0 + x];
          sM[2][x] = io.mom[4 * N + b0 + x];
          sM[3][x] = io.mom[5 * N + b0 + x];
        }
        sM[4][x] = io.q_iso ? io.q_iso[b0 + x] : 0.0;
      }
    }
    __syncthreads();
    int bad = 0;
    if (i < nvol) {
      const int e = i / Q, q = i % Q;
      const double *V = STAGE ? sV + q * n : pb.tab_d + (size_t)q * n;
      const int el = (e - e0) * n;  // the element's staged entries
      if (io.E && io.mom) {
        double ph = 0, pxx = 0, pxy = 0, pyy = 0;
        for (int j = 0; j < n; ++j) {
          const double v = V[j];
          if constexpr (STAGE) {
            ph += sM[0][el + j] * v;
            pxx += sM[1][el + j] * v;
            pxy += sM[2][el + j] * v;
            pyy += sM[3][el + j] * v;
          } else {
            ph += io.mom[(size_t)e * n + j] * v;
            pxx += io.mom[3 * N + (size_t)e * n + j] * v;
            pxy += io.mom[4 * N + (size_t)e * n + j] * v;
            pyy += io.mom[5 * N + (size_t)e * n + j] * v;
          }
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
          for (int j = 0; j < n; ++j) qi += (STAGE ? sM[4][el + j] : io.q_iso[(size_t)e * n + j]) * V[j];
        double s0 = 0, s1 = 0, s2 = 0;
        if (io.q_dir) {
          for (int d = 0; d < nd; ++d) {
            const double qq = qi + io.q_dir[((size_t)d * ne + e) * Q + q];
            s0 += dirs[d].x * qq;
            s1 += dirs[d].y * qq;
            s2 += dirs[d].z * qq;
          }
        } else {
          s0 = qi * wsum[0];
          s1 = qi * wsum[1];
          s2 = qi * wsum[2];
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
}

__global__ void k_zero_nonpos(const KMomIO *__restrict__ io, int n_probs) {
  const int i = threadIdx.x;
  if (i < n_probs && io[i].n_nonpos) *io[i].n_nonpos = 0;
}

}  // namespace

hipError_t launch_sweep_p1(const SweepLaunch &L, bool dir);
hipError_t launch_sweep_p2(const SweepLaunch &L, bool dir);
hipError_t launch_sweep_p3(const SweepLaunch &L, bool dir);
hipError_t launch_sweep_p4(const SweepLaunch &L, bool dir);

static hipError_t launch_sweep(const SweepLaunch &L, bool dir) {
  switch (L.p) {
    case 1: return launch_sweep_p1(L, dir);
    case 2: return launch_sweep_p2(L, dir);
    case 3: return launch_sweep_p3(L, dir);
    case 4: return launch_sweep_p4(L, dir);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_class_inv_p3(const ClassInvLaunch &C);
hipError_t launch_class_inv_p4(const ClassInvLaunch &C);

hipError_t launch_class_inv(const ClassInvLaunch &C) {
  switch (C.p) {
    case 3: return launch_class_inv_p3(C);
    case 4: return launch_class_inv_p4(C);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pivot_order_p3(const PivotOrderLaunch &L);

hipError_t launch_pivot_order(const PivotOrderLaunch &L) {
  return L.p == 3 ? launch_pivot_order_p3(L) : hipErrorInvalidValue;
}

hipError_t launch_sweep_level(const SweepLaunch &L) { return launch_sweep(L, false); }
hipError_t launch_sweep_dir(const SweepLaunch &L) { return launch_sweep(L, true); }

hipError_t launch_moments(bool fp32, const KProb *probs, const KIO *io, int prob, int ne_n, int nd, int it,
                          const int *stop, hipStream_t s) {
  if (nd < 1 || nd > kMaxMomDirs) return hipErrorInvalidValue;
  const int grid = (ne_n + 63) / 64;
  const size_t bytes = sizeof(double3) * (size_t)nd;
  if (fp32)
    hipLaunchKernelGGL(k_moments<float>, dim3(grid), dim3(64 * kMomWaves), bytes, s, probs, io, prob, ne_n, it,
                       stop);
  else
    hipLaunchKernelGGL(k_moments<double>, dim3(grid), dim3(64 * kMomWaves), bytes, s, probs, io, prob, ne_n, it,
                       stop);
  return hipGetLastError();
}

hipError_t launch_boundary(bool fp32, const KProb *probs, const KIO *io, int prob, int nbf, int nq,
                           int p, const int *stop, hipStream_t s) {
  if (nbf == 0) return hipSuccess;
  if (nq > kBndMaxNq || p > 4) return hipErrorInvalidValue;
  const int grid = (nbf + 3) / 4;  // one wave per boundary face
  if (fp32)
    hipLaunchKernelGGL(k_boundary<float>, dim3(grid), dim3(256), 0, s, probs, io, prob, nbf, nq, p, stop);
  else
    hipLaunchKernelGGL(k_boundary<double>, dim3(grid), dim3(256), 0, s, probs, io, prob, nbf, nq, p, stop);
  return hipGetLastError();
}

hipError_t launch_run_init(const KIO *io, int n_probs, int n_iter, int *stop, int *iters, int *status,
                           hipStream_t s) {
  const int tot = n_probs * n_iter;
  const int grid = (tot + 255) / 256 > 0 ? (tot + 255) / 256 : 1;
  hipLaunchKernelGGL(k_run_init, dim3(grid), dim3(256), 0, s, io, n_probs, n_iter, stop, iters, status);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_finalize(const KIO *io, int n_probs, int it, double tol, int *stop, int *iters,
                           int *iters_user, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, io, n_probs, it, tol, stop, iters, iters_user);
  return hipGetLastError();
}

hipError_t launch_closures(const KProb *probs, const KMomIO *io, int prob, int ne, int Q, int n, int nbf,
                           int nq, hipStream_t s) {
  const int tot = ne * Q + nbf * nq;
  // enough work-groups to fill the device a few times over; each loops over
  // its chunks
  const int need = (tot + kClThreads - 1) / kClThreads;
  const int grid = need < kClMaxGroups ? need : kClMaxGroups;
  // LDS staging when a work-group's elements and the basis table fit
  const bool stage = Q > 0 && (kClThreads / Q + 2) * n <= kClStageEl && Q * n <= kClStageV;
  if (stage)
    hipLaunchKernelGGL(k_closures<true>, dim3(grid), dim3(kClThreads), 0, s, probs, io, prob, ne, Q, nbf, nq);
  else
    hipLaunchKernelGGL(k_closures<false>, dim3(grid), dim3(kClThreads), 0, s, probs, io, prob, ne, Q, nbf, nq);
  return hipGetLastError();
}

hipError_t launch_zero_nonpos(const KMomIO *io, int n_probs, hipStream_t s) {
  // one thread per problem; n_probs is bounded by the handle (<= 1024)
  hipLaunchKernelGGL(k_zero_nonpos, dim3(1), dim3(1024), 0, s, io, n_probs);
  return hipGetLastError();
}

}  // namespace vefk

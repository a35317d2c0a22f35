// Direction-independent element matrices of general (curved) elements of
// degree 3 on the matrix cores.
//
// The transport operator on element K tested with phi_i (Sec. 3.2: the
// integrals are mapped to the reference square through the Jacobian and the
// adjugate of the element map; Sec. 5: one local system per element and
// direction) splits into parts that do not depend on the direction,
//   M_ij   = sum_q (w J)_q V_qi V_qj,
//   G^x_ij = sum_q [(w adj F)_00 Dx_qi + (w adj F)_10 Dy_qi]_q V_qj,
//   G^y_ij = sum_q [(w adj F)_01 Dx_qi + (w adj F)_11 Dy_qi]_q V_qj,
// (V, Dx, Dy: the basis and its reference derivatives at the Q volume
// points) so that the local matrix for a direction is sigma_t M - Omega_x G^x
// - Omega_y G^y plus face terms.  Each is a 16 x Q by Q x 16 product: one
// wave per element accumulates the three with v_mfma_f64_16x16x4 over Q in
// chunks of 4 points (zero padded), the B operand (V) shared by all three.
// The face matrices F^c_f[pos][k] = sum_s (w n_c ds)_s L_s,pos L_s,k (L the
// 1D basis at the face points) take one lane each.
//
// Layout per element: M, G^x, G^y, each with entry (i, j) at
// ((j / W) 16 + i) W + j % W, W = 16 bytes / sizeof(T) (so that the 16 lanes
// of a solve, lane i reading row i, read 16 W consecutive values per 16-byte
// load), then the face matrices [f][component][pos][k].

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vefk {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int NQ, typename T>
__global__ void __launch_bounds__(256) k_elem_mat(int ne, const double *__restrict__ tab, const double *__restrict__ gv,
                                                  const double *__restrict__ gf, T *__restrict__ out) {
  constexpr int P = 3, P1 = 4, N = 16, Q = NQ * NQ;
  constexpr int SIZE = 3 * N * N + 8 * P1 * P1;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;  // whole waves
  const int lane = threadIdx.x & 63;
  const double *V = tab, *Dx = tab + Q * N, *Dy = tab + 2 * Q * N, *F = tab + 3 * Q * N;
  const double *g = gv + (size_t)e * Q * 5;
  // operand layout of the 16x16x4 f64 product (checked on the device): A[i][k]
  // and B[k][j] in lane i + 16 k (j + 16 k); D[i][j] in lane j + 16 (i % 4),
  // element i / 4
  const int i = lane & 15, kk = lane >> 4;
  dbl4 m = {0.0, 0.0, 0.0, 0.0}, cx = m, cy = m;
#pragma unroll
  for (int k0 = 0; k0 < Q; k0 += 4) {
    const int q = k0 + kk;
    double am = 0.0, ax = 0.0, ay = 0.0, bv = 0.0;
    if (q < Q) {
      const double vq = V[q * N + i], dx = Dx[q * N + i], dy = Dy[q * N + i];
      const double wJ = g[5 * q], a00 = g[5 * q + 1], a01 = g[5 * q + 2], a10 = g[5 * q + 3], a11 = g[5 * q + 4];
      am = wJ * vq;
      ax = a00 * dx + a10 * dy;
      ay = a01 * dx + a11 * dy;
      bv = vq;
    }
    m = __builtin_amdgcn_mfma_f64_16x16x4f64(am, bv, m, 0, 0, 0);
    cx = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bv, cx, 0, 0, 0);
    cy = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, bv, cy, 0, 0, 0);
  }
  T *o = out + (size_t)e * SIZE;
  constexpr int W = 16 / sizeof(T);
  const int j = lane & 15;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = (lane >> 4) + 4 * v;
    const int at = ((j / W) * 16 + row) * W + j % W;
    o[at] = static_cast<T>(m[v]);
    o[N * N + at] = static_cast<T>(cx[v]);
    o[2 * N * N + at] = static_cast<T>(cy[v]);
  }
  // face matrices: lane = 16 f + 4 pos + k
  {
    const int f = lane >> 4, pos = (lane >> 2) & 3, k = lane & 3;
    const double *fg = gf + (size_t)e * 8 * NQ + f * 2 * NQ;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
      const double l2 = F[s * P1 + pos] * F[s * P1 + k];
      sx += fg[2 * s] * l2;
      sy += fg[2 * s + 1] * l2;
    }
    o[3 * N * N + (2 * f) * P1 * P1 + pos * P1 + k] = static_cast<T>(sx);
    o[3 * N * N + (2 * f + 1) * P1 * P1 + pos * P1 + k] = static_cast<T>(sy);
  }
  (void)P;
}

template <int NQ>
hipError_t launch_nq(bool fp32, int ne, const double *tab, const double *gv, const double *gf, void *out,
                     hipStream_t s) {
  const int block = 256, grid = (ne + 3) / 4;
  if (fp32)
    hipLaunchKernelGGL((k_elem_mat<NQ, float>), dim3(grid), dim3(block), 0, s, ne, tab, gv, gf,
                       static_cast<float *>(out));
  else
    hipLaunchKernelGGL((k_elem_mat<NQ, double>), dim3(grid), dim3(block), 0, s, ne, tab, gv, gf,
                       static_cast<double *>(out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_elem_mat(int p, int nq, bool fp32, int ne, const double *tab_d, const double *geo_vd,
                           const double *geo_fd, void *out, hipStream_t s) {
  if (p != 3 || ne <= 0) return hipErrorInvalidValue;
  switch (nq) {
    case 4: return launch_nq<4>(fp32, ne, tab_d, geo_vd, geo_fd, out, s);
    case 5: return launch_nq<5>(fp32, ne, tab_d, geo_vd, geo_fd, out, s);
    case 6: return launch_nq<6>(fp32, ne, tab_d, geo_vd, geo_fd, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vefk

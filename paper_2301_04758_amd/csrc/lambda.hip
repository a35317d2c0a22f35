// Device solve of the reduced hybridized system of Sec. 7: after the
// element-local elimination of [J; phi], the face unknowns lambda satisfy
// H lambda = r with H and r sums of element contributions over the
// interior-face slots of each element (Eq. eq:hyb_form with the element
// blocks eliminated).  The sparsity pattern of H depends only on the mesh,
// so one host factorisation P H0 Q = L U fixes the pivot order and the fill,
// and every later matrix of the outer iteration is re-factorised numerically
// on the device (rocSOLVER's csrrf routines: a library sparse LU, the same
// role a sparse direct solver plays for the paper's VEF solve).  Assembly,
// residual and the element-by-element recovery
// [J; phi] = sol0 - resp lambda_loc are kernels of this file.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "vef_sweep.h"

struct vef_lambda {
  int n = 0, ne = 0, k = 0, nloc = 0, nnz = 0, nnz_t = 0;
  int *ptr = nullptr, *ind = nullptr;        // CSR pattern of H
  int *ptr_t = nullptr, *ind_t = nullptr;    // pattern of T = (L - I) + U
  int *piv_p = nullptr, *piv_q = nullptr;
  double *val = nullptr, *val_t = nullptr;   // values of H and of T
  double *rhs = nullptr;                     // r (kept for the residual)
  int2 *src_h = nullptr;                     // per nonzero: up to two flat hloc indices (-1 none)
  int2 *src_r = nullptr;                     // per unknown: up to two flat rloc indices
  int *gidx = nullptr;                       // [ne][k]
  double *red = nullptr;                     // [4] residual reduction
  rocblas_handle blas = nullptr;
  rocsolver_rfinfo rf = nullptr;
  std::string err;
};

namespace {

std::string g_lambda_err;

int lam_err(vef_lambda *h, int code, const std::string &m) {
  if (h) h->err = m;
  else g_lambda_err = m;
  return code;
}

int lam_hip(vef_lambda *h, hipError_t e, const char *what) {
  return lam_err(h, e == hipErrorOutOfMemory ? VEF_ERR_OOM : VEF_ERR_HIP,
                 std::string(what) + ": " + hipGetErrorString(e));
}

__global__ void k_gather2(const int2 *__restrict__ src, int count, const double *__restrict__ a,
                          double *__restrict__ out, double *__restrict__ out2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int2 s = src[i];
  double v = 0.0;
  if (s.x >= 0) v += a[s.x];
  if (s.y >= 0) v += a[s.y];
  out[i] = v;
  if (out2) out2[i] = v;
}

// sol[e][r] = sol0[e][r] - sum_j resp[e][r][j] lambda[gidx[e][j]]
__global__ void k_recover(const double *__restrict__ sol0, const double *__restrict__ resp,
                          const int *__restrict__ gidx, const double *__restrict__ lam, double *__restrict__ sol,
                          int ne, int nloc, int k) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)ne * nloc) return;
  const int e = (int)(i / nloc);
  const double *rp = resp + i * k;
  const int *g = gidx + (size_t)e * k;
  double acc = sol0[i];
  for (int j = 0; j < k; ++j) {
    const int c = g[j];
    if (c >= 0) acc -= rp[j] * lam[c];
  }
  sol[i] = acc;
}

// Normwise backward error of lambda: out[0] = max_i |r_i - (H lambda)_i|,
// out[1] = max_i |r_i|, out[2] = max_i sum_j |H_ij|, out[3] = max_i |lambda_i|,
// as the bit patterns of non-negative doubles (whose unsigned order is their
// numeric order), so that work-groups combine by atomic max; out starts at 0.
__global__ void k_zero4(unsigned long long *out) {
  if (threadIdx.x < 4) out[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(256) k_residual(const int *__restrict__ ptr, const int *__restrict__ ind,
                                                  const double *__restrict__ val, const double *__restrict__ lam,
                                                  const double *__restrict__ rhs, int n,
                                                  unsigned long long *__restrict__ out) {
  __shared__ double s_m[4][256];
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double acc = rhs[i], rs = 0.0;
    for (int j = ptr[i]; j < ptr[i + 1]; ++j) {
      acc -= val[j] * lam[ind[j]];
      rs += fabs(val[j]);
    }
    m[0] = fabs(acc);
    m[1] = fabs(rhs[i]);
    m[2] = rs;
    m[3] = fabs(lam[i]);
  }
  for (int c = 0; c < 4; ++c) s_m[c][threadIdx.x] = m[c];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) s_m[c][threadIdx.x] = fmax(s_m[c][threadIdx.x], s_m[c][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 4) atomicMax(out + threadIdx.x, (unsigned long long)__double_as_longlong(s_m[threadIdx.x][0]));
}

template <typename X>
hipError_t put(X **d, const X *h, size_t n) {
  hipError_t e = hipMalloc(reinterpret_cast<void **>(d), std::max<size_t>(n, 1) * sizeof(X));
  if (e == hipSuccess && n) e = hipMemcpy(*d, h, n * sizeof(X), hipMemcpyHostToDevice);
  return e;
}

bool is_permutation(const int32_t *p, int n) {
  std::vector<char> seen(n, 0);
  for (int i = 0; i < n; ++i) {
    if (p[i] < 0 || p[i] >= n || seen[p[i]]) return false;
    seen[p[i]] = 1;
  }
  return true;
}

bool csr_ok(const int32_t *ptr, const int32_t *ind, int n, int nnz) {
  if (ptr[0] != 0 || ptr[n] != nnz) return false;
  for (int i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) return false;
    for (int j = ptr[i]; j < ptr[i + 1]; ++j) {
      if (ind[j] < 0 || ind[j] >= n) return false;
      if (j > ptr[i] && ind[j] <= ind[j - 1]) return false;
    }
  }
  return true;
}

hipError_t assemble(vef_lambda *h, const double *hloc, const double *rloc, double *b, hipStream_t s) {
  const int T = 256;
  hipLaunchKernelGGL(k_gather2, dim3((h->nnz + T - 1) / T), dim3(T), 0, s, h->src_h, h->nnz, hloc, h->val,
                     (double *)nullptr);
  hipLaunchKernelGGL(k_gather2, dim3((h->n + T - 1) / T), dim3(T), 0, s, h->src_r, h->n, rloc, h->rhs, b);
  return hipGetLastError();
}

}  // namespace

extern "C" {

const char *vef_lambda_error(const vef_lambda_t *h) { return h ? h->err.c_str() : g_lambda_err.c_str(); }

int vef_lambda_destroy(vef_lambda_t *h) {
  if (!h) return VEF_OK;
  if (h->rf) rocsolver_destroy_rfinfo(h->rf);
  if (h->blas) rocblas_destroy_handle(h->blas);
  for (void *p : {(void *)h->ptr, (void *)h->ind, (void *)h->ptr_t, (void *)h->ind_t, (void *)h->piv_p,
                  (void *)h->piv_q, (void *)h->val, (void *)h->val_t, (void *)h->rhs, (void *)h->src_h,
                  (void *)h->src_r, (void *)h->gidx, (void *)h->red})
    if (p) (void)hipFree(p);
  delete h;
  return VEF_OK;
}

int vef_lambda_create(int n, int ne, int k, int nloc, const int32_t *gidx, int nnz_t, const int32_t *ptr_t,
                      const int32_t *ind_t, const double *val_t, const int32_t *piv_p, const int32_t *piv_q,
                      const double *hloc0, const double *rloc0, void *stream, vef_lambda_t **out) {
  if (!out) return lam_err(nullptr, VEF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (n < 1 || ne < 1 || k < 1 || nloc < 1 || nnz_t < n || !gidx || !ptr_t || !ind_t || !val_t || !piv_p ||
      !piv_q || !hloc0 || !rloc0)
    return lam_err(nullptr, VEF_ERR_INVALID, "bad sizes or NULL arguments");
  if ((long long)ne * k * k >= (1LL << 31) || (long long)ne * nloc * k >= (1LL << 40))
    return lam_err(nullptr, VEF_ERR_INVALID, "element blocks too large for 32-bit indexing");
  for (long long i = 0; i < (long long)ne * k; ++i)
    if (gidx[i] < -1 || gidx[i] >= n) return lam_err(nullptr, VEF_ERR_INVALID, "gidx entry out of range");
  if (!csr_ok(ptr_t, ind_t, n, nnz_t)) return lam_err(nullptr, VEF_ERR_INVALID, "bad CSR pattern of T");
  if (!is_permutation(piv_p, n) || !is_permutation(piv_q, n))
    return lam_err(nullptr, VEF_ERR_INVALID, "piv_p and piv_q must be permutations of 0..n-1");
  // pattern of H: the (gidx[e][i], gidx[e][j]) pairs, and for each nonzero
  // the element entries that add into it (a face's diagonal block has the
  // two elements of the face, any other pair of faces at most one element)
  std::vector<std::vector<std::pair<int, int>>> rows(n);  // (col, flat hloc index)
  std::vector<int2> src_r(n, make_int2(-1, -1));
  for (int e = 0; e < ne; ++e)
    for (int i = 0; i < k; ++i) {
      const int gi = gidx[(size_t)e * k + i];
      if (gi < 0) continue;
      int2 &sr = src_r[gi];
      const int fl = e * k + i;
      if (sr.x < 0) sr.x = fl;
      else if (sr.y < 0) sr.y = fl;
      else return lam_err(nullptr, VEF_ERR_INVALID, "an unknown is shared by more than two elements");
      for (int j = 0; j < k; ++j) {
        const int gj = gidx[(size_t)e * k + j];
        if (gj >= 0) rows[gi].push_back({gj, (e * k + i) * k + j});
      }
    }
  std::vector<int32_t> ptr(n + 1, 0), ind;
  std::vector<int2> src_h;
  for (int i = 0; i < n; ++i) {
    auto &r = rows[i];
    std::sort(r.begin(), r.end());
    for (size_t a = 0; a < r.size();) {
      size_t b = a;
      int2 s = make_int2(r[a].second, -1);
      while (++b < r.size() && r[b].first == r[a].first) {
        if (s.y >= 0) return lam_err(nullptr, VEF_ERR_INVALID, "a nonzero of H has more than two contributions");
        s.y = r[b].second;
      }
      ind.push_back(r[a].first);
      src_h.push_back(s);
      a = b;
    }
    ptr[i + 1] = (int32_t)ind.size();
    std::vector<std::pair<int, int>>().swap(r);
  }
  vef_lambda *h = new vef_lambda;
  h->n = n;
  h->ne = ne;
  h->k = k;
  h->nloc = nloc;
  h->nnz = (int)ind.size();
  h->nnz_t = nnz_t;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t he = put(&h->ptr, ptr.data(), ptr.size());
  if (he == hipSuccess) he = put(&h->ind, ind.data(), ind.size());
  if (he == hipSuccess) he = put(&h->ptr_t, ptr_t, (size_t)n + 1);
  if (he == hipSuccess) he = put(&h->ind_t, ind_t, (size_t)nnz_t);
  if (he == hipSuccess) he = put(&h->val_t, val_t, (size_t)nnz_t);
  if (he == hipSuccess) he = put(&h->piv_p, piv_p, (size_t)n);
  if (he == hipSuccess) he = put(&h->piv_q, piv_q, (size_t)n);
  if (he == hipSuccess) he = put(&h->src_h, src_h.data(), src_h.size());
  if (he == hipSuccess) he = put(&h->src_r, src_r.data(), src_r.size());
  if (he == hipSuccess) he = put(&h->gidx, gidx, (size_t)ne * k);
  if (he == hipSuccess) he = hipMalloc(&h->val, (size_t)h->nnz * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&h->rhs, (size_t)n * sizeof(double));
  if (he == hipSuccess) he = hipMalloc(&h->red, 4 * sizeof(double));
  if (he != hipSuccess) {
    lam_hip(nullptr, he, "upload of the lambda system");
    vef_lambda_destroy(h);
    return he == hipErrorOutOfMemory ? VEF_ERR_OOM : VEF_ERR_HIP;
  }
  if (rocblas_create_handle(&h->blas) != rocblas_status_success ||
      rocblas_set_stream(h->blas, s) != rocblas_status_success ||
      rocsolver_create_rfinfo(&h->rf, h->blas) != rocblas_status_success) {
    vef_lambda_destroy(h);
    return lam_err(nullptr, VEF_ERR_HIP, "rocBLAS / rocSOLVER set-up failed");
  }
  // analysis with the matrix the factors were computed from
  double *b = nullptr;
  he = hipMalloc(&b, (size_t)n * sizeof(double));
  if (he == hipSuccess) he = assemble(h, hloc0, rloc0, b, s);
  if (he != hipSuccess) {
    if (b) (void)hipFree(b);
    lam_hip(nullptr, he, "assembly of H0");
    vef_lambda_destroy(h);
    return VEF_ERR_HIP;
  }
  const rocblas_status st = rocsolver_dcsrrf_analysis(h->blas, n, 1, h->nnz, h->ptr, h->ind, h->val, nnz_t, h->ptr_t,
                                                      h->ind_t, h->val_t, h->piv_p, h->piv_q, b, n, h->rf);
  he = hipStreamSynchronize(s);
  (void)hipFree(b);
  if (st != rocblas_status_success || he != hipSuccess) {
    vef_lambda_destroy(h);
    return lam_err(nullptr, VEF_ERR_HIP, "rocsolver_dcsrrf_analysis failed (status " + std::to_string((int)st) + ")");
  }
  *out = h;
  return VEF_OK;
}

int vef_lambda_solve(vef_lambda_t *h, const double *hloc, const double *rloc, const double *sol0, const double *resp,
                     double *lam, double *sol, double *rel_resid, void *stream) {
  if (!h) return VEF_ERR_INVALID;
  if (!hloc || !rloc || !lam || ((sol0 || resp || sol) && !(sol0 && resp && sol)))
    return lam_err(h, VEF_ERR_INVALID, "hloc, rloc and lam are required; sol0, resp and sol go together");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (rocblas_set_stream(h->blas, s) != rocblas_status_success)
    return lam_err(h, VEF_ERR_HIP, "rocblas_set_stream failed");
  hipError_t he = assemble(h, hloc, rloc, lam, s);
  if (he != hipSuccess) return lam_hip(h, he, "assembly of H");
  rocblas_status st = rocsolver_dcsrrf_refactlu(h->blas, h->n, h->nnz, h->ptr, h->ind, h->val, h->nnz_t, h->ptr_t,
                                                h->ind_t, h->val_t, h->piv_p, h->piv_q, h->rf);
  if (st == rocblas_status_success)
    st = rocsolver_dcsrrf_solve(h->blas, h->n, 1, h->nnz_t, h->ptr_t, h->ind_t, h->val_t, h->piv_p, h->piv_q, lam,
                                h->n, h->rf);
  if (st != rocblas_status_success)
    return lam_err(h, VEF_ERR_HIP, "rocSOLVER re-factorisation or solve failed (status " + std::to_string((int)st) + ")");
  if (sol) {
    const long long m = (long long)h->ne * h->nloc;
    hipLaunchKernelGGL(k_recover, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, sol0, resp, h->gidx, lam, sol,
                       h->ne, h->nloc, h->k);
    he = hipGetLastError();
    if (he != hipSuccess) return lam_hip(h, he, "launch recovery");
  }
  if (rel_resid) {
    auto *red = reinterpret_cast<unsigned long long *>(h->red);
    hipLaunchKernelGGL(k_zero4, dim3(1), dim3(64), 0, s, red);
    hipLaunchKernelGGL(k_residual, dim3((h->n + 255) / 256), dim3(256), 0, s, h->ptr, h->ind, h->val, lam, h->rhs,
                       h->n, red);
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    he = hipGetLastError();
    if (he == hipSuccess) he = hipMemcpyAsync(r, h->red, sizeof(r), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return lam_hip(h, he, "residual");
    const double scale = r[2] * r[3] + r[1];
    *rel_resid = scale > 0.0 ? r[0] / scale : r[0];
  }
  return VEF_OK;
}

}  // extern "C"

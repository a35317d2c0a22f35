// C ABI of the sweep library (declared in include/vef_sweep.h): handle
// creation (host plan + upload), runs (enqueue of the level-synchronous sweep,
// moment/residual/boundary kernels per source iteration), closures, queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "kernels.h"
#include "plan.h"
#include "vef_sweep.h"

namespace {

thread_local std::string g_create_error;

struct TableSet {
  void *dev_T = nullptr;       // float or double tables for the general sweep kernels
  void *dev_A = nullptr;       // float or double tables for the affine sweep kernels
  double *dev_d = nullptr;     // double tables for reductions / closures
};

// Kernel variant of a problem: degree, quadrature, assembly/solve mode
// (0: general elements with pivoting, 1: general pivot-free, 2: affine pivot-free).
struct Variant {
  int p, nq, mode;
  bool operator<(const Variant &o) const {
    return p != o.p ? p < o.p : (nq != o.nq ? nq < o.nq : mode < o.mode);
  }
};

int mode_of(const vefplan::ProblemPlan &pl, int schedule, bool pipeline = true, bool fixup = false) {
  if (pl.elem_mat) return 6;  // general elements, p = 3, precomputed element matrices
  if (!pl.nopivot) return 0;
  const bool pipe = pipeline && schedule == VEF_DIR_RESIDENT && pl.p <= 2;
  // straight-sided bilinear elements: the pipelined kernel with quadrature
  // assembly (lagged couplings read the previous sweep from global memory)
  (void)fixup;
  if (!pl.affine) return (pipe && pl.m == 1) ? 4 : 1;
  if (pl.p >= 3) return 5;  // row-set LU with fused broadcasts
  return (pipe && pl.n_lagged == 0) ? 3 : 2;
}

struct LevelLaunch {
  Variant v;
  int off, cnt;
  const void *tab;
  bool flow;  // its problems run in persistent launches under VEF_PERSISTENT
};

struct FlowLaunch {  // one persistent launch: the tasks of a variant (row-per-lane or row-set LU modes)
  Variant v;
  int off, cnt;  // into d_flow_tasks (off is also the flag index of the first task)
  const void *tab;
};

// Modes whose kernels stage the affine table blob (reference matrices);
// the others stage the quadrature tables (V, Dx, Dy, F).
bool affine_tables(int mode) { return mode >= 2 && mode <= 5; }

// Modes with a persistent kernel (no fixup variant).
bool flow_mode(int mode, int fixup) { return !fixup && (mode == 0 || mode == 1 || mode == 5 || mode == 6); }

// Kernel mode a launch of variant mode `mode` runs with: problems built for
// the element-matrix kernel (6) take the quadrature kernel with per-solve
// pivoting (0) when the handle's autotuner chose it; the two use the same
// lists, tables and slot shape.
int launch_mode(bool mat_quadrature, int mode) { return (mode == 6 && mat_quadrature) ? 0 : mode; }

// Solves per round of one wave of a kernel mode: 16-lane slots for the
// row-set LU, otherwise the power-of-two slot >= n of the row-per-lane kernels.
int solves_per_round(int mode, int n) {
  if (mode == 5) return 4;
  return 64 / (n <= 4 ? 4 : (n <= 8 ? 8 : (n <= 16 ? 16 : 32)));
}
constexpr int kFlowRounds = 2;  // rounds of solves per persistent task

struct DirLaunch {  // one direction-resident launch: all (problem, direction) pairs of a variant
  Variant v;
  int off, cnt;    // into d_dir_tasks
  int width;       // widest upwind level among the variant's problems
  int max_levels;  // deepest level count among them
  int max_gap;     // largest upwind level gap among them
  const void *tab;
  const void *tab_g;  // general tables of (p, nq)
};

}  // namespace

struct vef_sweep {
  std::string err;
  int precision = VEF_FP64;
  int schedule = VEF_SCHEDULE_AUTO;
  int block = 256;
  int device = 0;
  size_t lds_max = 65536;  // shared memory per work-group of the device
  std::vector<vefplan::ProblemPlan> plans;
  std::vector<void *> allocs;
  std::map<std::pair<int, int>, TableSet> tables;
  std::vector<vefk::KProb> h_probs;
  vefk::KProb *d_probs = nullptr;
  vefk::KIO *d_io = nullptr;
  vefk::KMomIO *d_mio = nullptr;
  vefk::KIO *h_io_pinned = nullptr;       // staging for d_io uploads
  vefk::KMomIO *h_mio_pinned = nullptr;   // staging for d_mio uploads
  hipEvent_t io_uploaded = nullptr;
  hipEvent_t mio_uploaded = nullptr;
  std::vector<vefk::KIO> io_last;
  bool io_valid = false;
  std::vector<vefk::KMomIO> mio_last;
  bool mio_valid = false;
  int2 *d_solves = nullptr;
  int4 *d_solve_desc = nullptr;  // per entry of d_solves: (element, direction | problem << 16, flags, class or
                                 // pivot-order entry), neighbours
  std::vector<std::vector<LevelLaunch>> levels;
  int2 *d_dir_tasks = nullptr;
  std::vector<FlowLaunch> flow;   // persistent schedule
  int2 *d_flow_tasks = nullptr;   // [n_flow_tasks] (first solve, solves)
  int *d_pred_ptr = nullptr;      // [n_flow_tasks + 1]
  int *d_pred_idx = nullptr;      // predecessor tasks of each task
  int *d_flow_flags = nullptr;    // [n_flow_tasks + 1]: sweep number per task, then the abort flag
  int n_flow_tasks = 0;
  int n_cu = 0;
  std::vector<DirLaunch> dir_rows;  // direction-resident, row-per-lane kernels only
  std::vector<DirLaunch> dir_pipe;  // direction-resident, pipelined kernel where it applies
  std::vector<void *> psi_internal;   // per problem, allocated on first need
  std::vector<double *> resid_scratch;
  std::vector<int> resid_cap;
  int *d_flags = nullptr;  // [0] stop, [1] iterations done, [2] status
  long long wait_polls = 1LL << 26;  // bound of one device-side wait (polls)
  bool elem_matrices = true;         // precomputed element matrices where available
  bool mat_quadrature = false;       // run-time choice (autotune): their problems take the quadrature kernel
  bool shared_matrices = true;       // classes of shared local matrices where a problem has them
  bool shared_lu = false;            // run-time choice (autotune): the row-set LU instead of the class matrices
  int n_cls = 0;                     // classes of shared local matrices of problem 0 (0: none)
  int4 *d_cls_rep = nullptr;         // [n_cls] representative (element, direction, inflow faces, 0)
  void *d_cls_inv = nullptr;         // T [n_cls][ncol][16][RS] class matrices (written by every run)
  double *static_resid = nullptr;    // this device's copy of `scratch` (vef_sweep_run_static)
  hipStream_t last_stream = nullptr;
  bool timing = false;
  int timing_stride = 0;  // time every timing_stride-th source iteration (and the last)
  int pipeline_waves = 0;
  int pipeline_ring = 0;
  int fixup = 0;
  int cycles = VEF_CYCLES_REJECT;
  int upwind = VEF_UPWIND_FACE;
  std::vector<double *> hrt_geo;               // per problem [ne][13], allocated on first need
  std::map<std::pair<int, int>, double *> hrt_tab;  // (p, nq) -> HRT tables
  std::vector<hipEvent_t> events;  // [2 * iterations] of the last run
  int timed_iters = 0;
  int timed_launches = 0;
};

// Per-sweep residuals of runs whose caller passes no residual buffer, for
// vef_sweep_run_static (no allocation in that call).  One copy per GPU, held
// until the process ends; every handle and call on that GPU shares it.  Host
// code never passes the array's name to a kernel: it uses the device address
// returned by hipGetSymbolAddress for the device that is current.
static __device__ __align__(256) double scratch[VEF_STATIC_RESID_MAX];

namespace {

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_addr;  // device -> address of its `scratch`

// Address of `scratch` on `device`, which must be the current device; looked
// up once per device.
hipError_t static_scratch_address(int device, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    it = g_scratch_addr.emplace(device, static_cast<double *>(ptr)).first;
  }
  *out = it->second;
  return hipSuccess;
}

int set_err(vef_sweep *h, int code, const std::string &msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return code;
}

int hip_fail(vef_sweep *h, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_err(h, e == hipErrorOutOfMemory ? VEF_ERR_OOM : VEF_ERR_HIP, m);
}

template <typename X>
hipError_t dev_alloc(vef_sweep *h, X **p, size_t count) {
  void *v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count * sizeof(X), 16));
  if (e != hipSuccess) return e;
  h->allocs.push_back(v);
  *p = static_cast<X *>(v);
  return hipSuccess;
}

template <typename X>
hipError_t upload(vef_sweep *h, X **p, const X *src, size_t count) {
  hipError_t e = dev_alloc(h, p, count);
  if (e != hipSuccess) return e;
  if (count == 0) return hipSuccess;
  return hipMemcpy(*p, src, count * sizeof(X), hipMemcpyHostToDevice);
}

template <typename X>
hipError_t upload_as(vef_sweep *h, void **p, const std::vector<double> &src) {
  std::vector<X> tmp(src.begin(), src.end());
  X *q = nullptr;
  hipError_t e = upload(h, &q, tmp.data(), tmp.size());
  *p = q;
  return e;
}

void free_all(vef_sweep *h) {
  if (!h) return;
  for (void *p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (void *p : h->psi_internal)
    if (p) (void)hipFree(p);
  h->psi_internal.clear();
  for (double *p : h->hrt_geo)
    if (p) (void)hipFree(p);
  h->hrt_geo.clear();
  for (auto &kv : h->hrt_tab) (void)hipFree(kv.second);
  h->hrt_tab.clear();
  for (double *p : h->resid_scratch)
    if (p) (void)hipFree(p);
  h->resid_scratch.clear();
  if (h->h_io_pinned) (void)hipHostFree(h->h_io_pinned);
  if (h->h_mio_pinned) (void)hipHostFree(h->h_mio_pinned);
  h->h_io_pinned = nullptr;
  h->h_mio_pinned = nullptr;
  for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
  h->events.clear();
  if (h->io_uploaded) (void)hipEventDestroy(h->io_uploaded);
  if (h->mio_uploaded) (void)hipEventDestroy(h->mio_uploaded);
  h->io_uploaded = h->mio_uploaded = nullptr;
}

std::vector<double> table_blob(const vefplan::Tables &t) {
  std::vector<double> b;
  b.insert(b.end(), t.V.begin(), t.V.end());
  b.insert(b.end(), t.Dx.begin(), t.Dx.end());
  b.insert(b.end(), t.Dy.begin(), t.Dy.end());
  b.insert(b.end(), t.F.begin(), t.F.end());
  return b;
}

// Classes of (direction, element) pairs that share one local matrix (row-set
// LU problems): on affine elements the matrix depends only on sigma_t, the
// element's J, adj(F) and face chords, the direction and which faces are
// inflow.  Element classes group equal bit patterns of the first four;
// solve classes add the direction and the inflow faces.
struct SharedClasses {
  int nd = 0, n_cls = 0;
  std::vector<int> ecls;  // [ne] element class
  std::vector<int> tab;   // [n_ecls][nd][16] solve class, or -1
  std::vector<int4> rep;  // [n_cls] (element, direction, inflow faces, 0)
  int of(const vefplan::ProblemPlan &pl, int e, int d) const {
    return tab[((size_t)ecls[e] * nd + d) * 16 + (pl.mask[(size_t)d * pl.ne + e] & 15u)];
  }
};

// Entries of one class matrix (kernels.h ClassInvLaunch): [ncol][16][RS].
size_t class_matrix_entries(const vefplan::ProblemPlan &pl) {
  const int tw = std::max(pl.p + 1, pl.nq);
  return (size_t)(pl.n + 8 * tw + pl.nq * pl.nq) * 16 * ((pl.n + 15) / 16);
}

constexpr int kMaxElemClasses = 4096;
constexpr int kMinSolvesPerClass = 8;
constexpr size_t kMaxClassInvBytes = size_t(16) << 20;

// True when the problem has few enough classes for the class matrices to pay
// (inv_bytes: bytes of one class matrix).
bool find_shared_classes(const vefplan::ProblemPlan &pl, size_t inv_bytes, SharedClasses &sc) {
  if (!pl.affine || pl.geo_a.size() != (size_t)pl.ne * 16) return false;
  std::map<std::array<uint64_t, 14>, int> keys;
  sc.ecls.assign(pl.ne, 0);
  for (int e = 0; e < pl.ne; ++e) {
    std::array<uint64_t, 14> k;
    std::memcpy(&k[0], &pl.sigma_t[e], sizeof(double));
    std::memcpy(&k[1], &pl.geo_a[(size_t)e * 16], 13 * sizeof(double));
    auto it = keys.emplace(k, (int)keys.size()).first;
    sc.ecls[e] = it->second;
    if ((int)keys.size() > kMaxElemClasses) return false;
  }
  if (keys.size() * (size_t)pl.nd * 16 > (size_t(1) << 24)) return false;
  sc.nd = pl.nd;
  sc.tab.assign(keys.size() * pl.nd * 16, -1);
  sc.rep.clear();
  for (int d = 0; d < pl.nd; ++d)
    for (int e = 0; e < pl.ne; ++e) {
      const unsigned m = pl.mask[(size_t)d * pl.ne + e] & 15u;
      int &c = sc.tab[((size_t)sc.ecls[e] * pl.nd + d) * 16 + m];
      if (c >= 0) continue;
      c = (int)sc.rep.size();
      sc.rep.push_back(make_int4(e, d, (int)m, 0));
    }
  sc.n_cls = (int)sc.rep.size();
  return (long long)sc.n_cls * kMinSolvesPerClass <= (long long)pl.ne * pl.nd &&
         (size_t)sc.n_cls * inv_bytes <= kMaxClassInvBytes;
}

int create_impl(const vef_problem_desc *probs, int n_probs, const vef_options *opt, vef_sweep *h) {
  if (opt) {
    if (opt->precision != VEF_FP64 && opt->precision != VEF_FP32_LOCAL)
      return set_err(h, VEF_ERR_INVALID, "unknown precision");
    if (opt->schedule != VEF_SCHEDULE_AUTO && opt->schedule != VEF_LEVEL_SYNC &&
        opt->schedule != VEF_DIR_RESIDENT && opt->schedule != VEF_PERSISTENT)
      return set_err(h, VEF_ERR_INVALID, "unknown schedule");
    if (opt->block != 0 && (opt->block < 64 || opt->block > 1024 || opt->block % 64))
      return set_err(h, VEF_ERR_INVALID, "block must be a multiple of 64 in 64..1024");
    h->precision = opt->precision;
    h->schedule = opt->schedule;
    if (opt->timing < 0) return set_err(h, VEF_ERR_INVALID, "timing must be >= 0");
    h->timing = opt->timing != 0;
    h->timing_stride = opt->timing;
    if (opt->pipeline_waves < -1 || opt->pipeline_waves > 8)
      return set_err(h, VEF_ERR_INVALID, "pipeline_waves must be -1..8");
    h->pipeline_waves = opt->pipeline_waves;
    if (opt->pipeline_ring < 0 || opt->pipeline_ring > 4)
      return set_err(h, VEF_ERR_INVALID, "pipeline_ring must be 0..4");
    h->pipeline_ring = opt->pipeline_ring;
    if (opt->fixup < 0 || opt->fixup > 1) return set_err(h, VEF_ERR_INVALID, "fixup must be 0 or 1");
    h->fixup = opt->fixup;
    if (opt->cycles != VEF_CYCLES_REJECT && opt->cycles != VEF_CYCLES_LAG)
      return set_err(h, VEF_ERR_INVALID, "cycles must be VEF_CYCLES_REJECT or VEF_CYCLES_LAG");
    h->cycles = opt->cycles;
    if (opt->upwind != VEF_UPWIND_FACE && opt->upwind != VEF_UPWIND_POINT)
      return set_err(h, VEF_ERR_INVALID, "unknown upwind rule");
    if (opt->upwind == VEF_UPWIND_POINT && opt->fixup)
      return set_err(h, VEF_ERR_INVALID, "the fixup is not available with pointwise upwinding");
    h->upwind = opt->upwind;
    if (opt->wait_polls < 0) return set_err(h, VEF_ERR_INVALID, "wait_polls must be >= 0");
    if (opt->wait_polls > 0) h->wait_polls = opt->wait_polls;
    if (opt->elem_matrices != 0 && opt->elem_matrices != -1)
      return set_err(h, VEF_ERR_INVALID, "elem_matrices must be 0 or -1");
    h->elem_matrices = opt->elem_matrices == 0;
    if (opt->shared_matrices != 0 && opt->shared_matrices != -1)
      return set_err(h, VEF_ERR_INVALID, "shared_matrices must be 0 or -1");
    h->shared_matrices = opt->shared_matrices == 0;
    h->block = opt->block ? opt->block : 256;
    if (h->block > 256) h->block = 256;  // kernels are built for at most 256 threads
  }
  if (n_probs > 1024) return set_err(h, VEF_ERR_INVALID, "at most 1024 problems per handle");
  h->plans.resize(n_probs);
  for (int k = 0; k < n_probs; ++k) {
    std::string e;
    int rc = vefplan::build_problem_plan(probs[k], h->cycles == VEF_CYCLES_LAG, h->upwind == VEF_UPWIND_POINT,
                                         h->plans[k], e);
    if (rc) return set_err(h, rc, "problem " + std::to_string(k) + ": " + e);
    auto &pl = h->plans[k];
    pl.elem_mat = h->elem_matrices && !pl.affine && pl.p == 3 && h->upwind == VEF_UPWIND_FACE;
  }
  hipError_t he = hipGetDevice(&h->device);
  if (he != hipSuccess) return hip_fail(h, he, "hipGetDevice");
  he = static_scratch_address(h->device, &h->static_resid);
  if (he != hipSuccess) return hip_fail(h, he, "hipGetSymbolAddress of the static residual array");
  int lds = 0;
  he = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
  if (he != hipSuccess) return hip_fail(h, he, "hipDeviceGetAttribute");
  h->lds_max = (size_t)lds;
  he = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device);
  if (he != hipSuccess) return hip_fail(h, he, "hipDeviceGetAttribute");
  const bool fp32 = h->precision == VEF_FP32_LOCAL;

  // tables per (p, nq)
  for (auto &pl : h->plans) {
    auto key = std::make_pair(pl.p, pl.nq);
    if (h->tables.count(key)) continue;
    TableSet ts;
    std::vector<double> blob = table_blob(pl.tab);
    he = fp32 ? upload_as<float>(h, &ts.dev_T, blob) : upload_as<double>(h, &ts.dev_T, blob);
    if (he == hipSuccess)
      he = fp32 ? upload_as<float>(h, &ts.dev_A, pl.tab.affine) : upload_as<double>(h, &ts.dev_A, pl.tab.affine);
    if (he != hipSuccess) return hip_fail(h, he, "upload tables");
    he = upload(h, &ts.dev_d, blob.data(), blob.size());
    if (he != hipSuccess) return hip_fail(h, he, "upload tables");
    h->tables[key] = ts;
  }

  // classes of shared local matrices (one-problem handles, row-set LU)
  SharedClasses shared;
  if (h->shared_matrices && n_probs == 1 && mode_of(h->plans[0], VEF_LEVEL_SYNC) == 5) {
    const auto &pl = h->plans[0];
    const size_t per = class_matrix_entries(pl);
    if (find_shared_classes(pl, per * (fp32 ? sizeof(float) : sizeof(double)), shared)) {
      h->n_cls = shared.n_cls;
      he = upload(h, &h->d_cls_rep, shared.rep.data(), shared.rep.size());
      if (he == hipSuccess)
        he = fp32 ? dev_alloc(h, reinterpret_cast<float **>(&h->d_cls_inv), (size_t)h->n_cls * per)
                  : dev_alloc(h, reinterpret_cast<double **>(&h->d_cls_inv), (size_t)h->n_cls * per);
      if (he != hipSuccess) return hip_fail(h, he, "allocate class matrices");
    }
  }

  // per-problem constant data
  h->h_probs.resize(n_probs);
  // per problem: d ne + e -> its entry of piv_perm (needed only while the
  // descriptors below are built)
  std::vector<std::unordered_map<long long, int>> piv_index(n_probs);
  std::vector<std::vector<int2>> piv_lists(n_probs);  // (element, direction) of the uncertified solves
  for (int k = 0; k < n_probs; ++k) {
    const auto &pl = h->plans[k];
    vefk::KProb kp{};
    kp.ne = pl.ne;
    kp.nd = pl.nd;
    kp.nbf = pl.nbf;
    kp.n = pl.n;
    kp.Q = pl.Q;
    kp.nq = pl.nq;
    kp.p = pl.p;
    kp.pointwise = h->upwind == VEF_UPWIND_POINT ? 1 : 0;
    void *gv = nullptr, *gf = nullptr;
    he = fp32 ? upload_as<float>(h, &gv, pl.geo_v) : upload_as<double>(h, &gv, pl.geo_v);
    if (he == hipSuccess) he = fp32 ? upload_as<float>(h, &gf, pl.geo_f) : upload_as<double>(h, &gf, pl.geo_f);
    kp.geo_v = gv;
    kp.geo_f = gf;
    void *ga = nullptr;
    if (he == hipSuccess && pl.affine)
      he = fp32 ? upload_as<float>(h, &ga, pl.geo_a) : upload_as<double>(h, &ga, pl.geo_a);
    kp.geo_a = ga;
    double *gfd = nullptr, *om = nullptr, *wt = nullptr, *sig = nullptr, *bnd = nullptr;
    int32_t *nbr = nullptr, *bfe = nullptr;
    int8_t *nbf = nullptr;
    uint8_t *mask = nullptr;
    std::vector<double> sg(2 * (size_t)pl.ne);
    for (int e = 0; e < pl.ne; ++e) {
      sg[2 * e] = pl.sigma_t[e];
      sg[2 * e + 1] = pl.sigma_s[e];
    }
    if (he == hipSuccess) he = upload(h, &gfd, pl.geo_f.data(), pl.geo_f.size());
    if (he == hipSuccess) he = upload(h, &nbr, pl.nbr.data(), pl.nbr.size());
    if (he == hipSuccess) he = upload(h, &nbf, pl.nbr_face.data(), pl.nbr_face.size());
    if (he == hipSuccess) he = upload(h, &mask, pl.mask.data(), pl.mask.size());
    if (he == hipSuccess) he = upload(h, &om, pl.omega.data(), pl.omega.size());
    if (he == hipSuccess) he = upload(h, &wt, pl.weight.data(), pl.weight.size());
    if (he == hipSuccess) he = upload(h, &sig, sg.data(), sg.size());
    if (he == hipSuccess) he = upload(h, &bfe, pl.bf_ef.data(), pl.bf_ef.size());
    if (he == hipSuccess) he = dev_alloc(h, &bnd, (size_t)pl.nbf * pl.nq * 2);
    int32_t *dg = nullptr, *nlg = nullptr, *lof = nullptr, *ord = nullptr, *def = nullptr, *dnb = nullptr;
    uint32_t *dup = nullptr;
    if (he == hipSuccess) he = upload(h, &dup, pl.desc_up.data(), pl.desc_up.size());
    if (he == hipSuccess) he = upload(h, &def, pl.desc_ef.data(), pl.desc_ef.size());
    if (he == hipSuccess) he = upload(h, &dnb, pl.desc_nb.data(), pl.desc_nb.size());
    if (he == hipSuccess) he = upload(h, &dg, pl.dir_group.data(), pl.dir_group.size());
    if (he == hipSuccess) he = upload(h, &nlg, pl.n_levels_g.data(), pl.n_levels_g.size());
    if (he == hipSuccess) he = upload(h, &lof, pl.level_off.data(), pl.level_off.size());
    if (he == hipSuccess) he = upload(h, &ord, pl.order.data(), pl.order.size());
    if (he != hipSuccess) return hip_fail(h, he, "upload problem data");
    kp.dir_group = dg;
    kp.n_levels_g = nlg;
    kp.level_off = lof;
    kp.order = ord;
    kp.desc_ef = reinterpret_cast<const int2 *>(def);
    kp.desc_nb = reinterpret_cast<const int4 *>(dnb);
    kp.desc_up = dup;
    kp.n_levels = pl.n_levels;
    kp.n_groups = pl.n_groups;
    kp.geo_fd = gfd;
    kp.nbr = nbr;
    kp.nbr_face = nbf;
    kp.mask = mask;
    kp.omega = om;
    kp.weight = wt;
    kp.sig = sig;
    kp.bf_ef = bfe;
    kp.bnd = bnd;
    kp.tab_d = h->tables[std::make_pair(pl.p, pl.nq)].dev_d;
    if (pl.elem_mat) {
      // direction-independent element matrices, formed once from double
      // geometry (a temporary double copy of the volume geometry for float)
      const size_t per = 3 * (size_t)pl.n * pl.n + 8 * (size_t)(pl.p + 1) * (pl.p + 1);
      void *em = nullptr;
      he = fp32 ? dev_alloc(h, reinterpret_cast<float **>(&em), per * pl.ne)
                : dev_alloc(h, reinterpret_cast<double **>(&em), per * pl.ne);
      const double *gvd = static_cast<const double *>(gv);
      double *tmp = nullptr;
      if (he == hipSuccess && fp32) {
        he = hipMalloc((void **)&tmp, sizeof(double) * pl.geo_v.size());
        if (he == hipSuccess)
          he = hipMemcpy(tmp, pl.geo_v.data(), sizeof(double) * pl.geo_v.size(), hipMemcpyHostToDevice);
        gvd = tmp;
      }
      if (he == hipSuccess) he = vefk::launch_elem_mat(pl.p, pl.nq, fp32, pl.ne, kp.tab_d, gvd, gfd, em, 0);
      if (he == hipSuccess) he = hipDeviceSynchronize();
      if (tmp) {
        const hipError_t fe = hipFree(tmp);
        if (he == hipSuccess) he = fe;
      }
      if (he != hipSuccess) return hip_fail(h, he, "element matrices");
      kp.emat = em;
      if (!pl.nopivot && pl.n_pivoting > 0) {
        // solves not certified for elimination in natural order: their row
        // order of partial pivoting, formed on the device below (by
        // direction, then element; the level lists carry the entry)
        auto &ix = piv_index[k];
        auto &ls = piv_lists[k];
        for (int d = 0; d < pl.nd; ++d)
          for (int e = 0; e < pl.ne; ++e)
            if (pl.mask[(size_t)d * pl.ne + e] & 0x80) {
              ix[(long long)d * pl.ne + e] = (int)ls.size();
              ls.push_back(make_int2(e, d));
            }
        uint8_t *pp = nullptr;
        he = dev_alloc(h, &pp, ls.size() * 16);
        if (he != hipSuccess) return hip_fail(h, he, "pivot orders");
        kp.piv_perm = pp;
      }
    }
    kp.cls_inv = h->n_cls > 0 ? h->d_cls_inv : nullptr;
    h->h_probs[k] = kp;
  }
  he = upload(h, &h->d_probs, h->h_probs.data(), h->h_probs.size());
  if (he != hipSuccess) return hip_fail(h, he, "upload problem records");
  for (int k = 0; k < n_probs; ++k) {
    if (piv_lists[k].empty()) continue;
    int2 *tmp = nullptr;
    vefk::PivotOrderLaunch PL{};
    PL.p = h->plans[k].p;
    PL.fp32 = fp32;
    PL.n = (int)piv_lists[k].size();
    PL.probs = h->d_probs;
    PL.prob = k;
    PL.out = const_cast<uint8_t *>(h->h_probs[k].piv_perm);
    he = hipMalloc((void **)&tmp, sizeof(int2) * piv_lists[k].size());
    if (he != hipSuccess) return hip_fail(h, he, "pivot orders");
    he = hipMemcpy(tmp, piv_lists[k].data(), sizeof(int2) * piv_lists[k].size(), hipMemcpyHostToDevice);
    PL.list = tmp;
    if (he == hipSuccess) he = vefk::launch_pivot_order(PL);
    if (he == hipSuccess) he = hipDeviceSynchronize();
    const hipError_t fe = hipFree(tmp);
    if (he == hipSuccess) he = fe;
    if (he != hipSuccess) return hip_fail(h, he, "pivot orders");
  }
  if (he == hipSuccess) he = dev_alloc(h, &h->d_io, n_probs);
  if (he == hipSuccess) he = dev_alloc(h, &h->d_mio, n_probs);
  if (he == hipSuccess) he = dev_alloc(h, &h->d_flags, 4);
  if (he == hipSuccess) he = hipMemset(h->d_flags, 0, 4 * sizeof(int));
  if (he == hipSuccess) he = hipHostMalloc((void **)&h->h_io_pinned, sizeof(vefk::KIO) * n_probs, 0);
  if (he == hipSuccess) he = hipHostMalloc((void **)&h->h_mio_pinned, sizeof(vefk::KMomIO) * n_probs, 0);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&h->io_uploaded, hipEventDisableTiming);
  if (he == hipSuccess) he = hipEventCreateWithFlags(&h->mio_uploaded, hipEventDisableTiming);
  if (he != hipSuccess) return hip_fail(h, he, "allocate handle buffers");

  if (h->schedule == VEF_SCHEDULE_AUTO) {
    // Direction-resident when every problem is narrow enough, level-synchronous
    // otherwise.  A level-synchronous level costs a launch (several us) however
    // narrow it is; a direction-resident level costs the work of the level on
    // one CU.  Measured crossovers: the row-per-lane kernel wins while the mean
    // level width fits in one round of slots of a work-group; the pipelined
    // kernel (about 1 us + 0.03 us per element of a level, p <= 2) up to a
    // mean width of about 256.
    bool narrow = true;
    for (auto &pl : h->plans) {
      const double width = (double)pl.ne / pl.n_levels;
      const int md = mode_of(pl, VEF_DIR_RESIDENT, h->pipeline_waves >= 0, h->fixup);
      if (md >= 3 && md <= 5) {
        if (width > 256.0) narrow = false;
        continue;
      }
      const int slot = pl.n <= 4 ? 4 : (pl.n <= 8 ? 8 : (pl.n <= 16 || (pl.affine && pl.p >= 3) ? 16 : 32));
      const int slots = (fp32 ? 1024 : 512) / slot;
      if (width > slots) narrow = false;
    }
    h->schedule = narrow ? VEF_DIR_RESIDENT : VEF_LEVEL_SYNC;
  }
  // level lists: level -> variant (p, nq) -> problem -> class -> element -> direction
  int max_levels = 0;
  for (auto &pl : h->plans) max_levels = std::max(max_levels, pl.n_levels);
  // Launch lists for every schedule are built here, so that the schedule and
  // the kernel can change after create (vef_sweep_autotune).
  std::vector<Variant> variants;
  {
    std::map<Variant, int> vs;
    for (auto &pl : h->plans) {
      vs[Variant{pl.p, pl.nq, mode_of(pl, VEF_DIR_RESIDENT, false)}] = 1;
      vs[Variant{pl.p, pl.nq, mode_of(pl, VEF_DIR_RESIDENT, true, h->fixup)}] = 1;
    }
    for (auto &kv : vs) variants.push_back(kv.first);
  }
  // the level-synchronous lists use the row-per-lane variant of every problem
  auto in_level_variant = [&](const vefplan::ProblemPlan &pl, const Variant &v) {
    const int m = mode_of(pl, VEF_LEVEL_SYNC);
    return pl.p == v.p && pl.nq == v.nq && m == v.mode;
  };
  std::vector<std::vector<std::vector<int>>> dirs_of(n_probs);
  for (int k = 0; k < n_probs; ++k) {
    const auto &pl = h->plans[k];
    dirs_of[k].resize(pl.n_groups);
    for (int d = 0; d < pl.nd; ++d) dirs_of[k][pl.dir_group[d]].push_back(d);
  }
  size_t total = 0;
  for (auto &pl : h->plans) total += (size_t)pl.ne * pl.nd;
  std::vector<int2> solves;
  solves.reserve(total);
  h->levels.assign(max_levels, {});
  // persistent schedule: tasks of kFlowRounds rounds of consecutive solves of
  // one (problem, class, level) block, per variant in level order; problems
  // with lagged couplings stay level-synchronous (a lagged read must precede
  // the re-solve of its upwind element, which only the level order enforces)
  std::vector<int> blk_first(n_probs, 0);
  int n_blk = 0;
  for (int k = 0; k < n_probs; ++k) {
    blk_first[k] = n_blk;
    n_blk += h->plans[k].n_groups * h->plans[k].n_levels;
  }
  std::vector<int> blk_solve0(n_blk, -1), blk_task0(n_blk, -1);
  std::map<Variant, std::vector<int2>> flow_tasks;
  std::map<Variant, std::vector<int>> flow_task_blk;
  auto flow_ok = [&](const vefplan::ProblemPlan &pl, const Variant &v) {
    return flow_mode(v.mode, h->fixup) && pl.n_lagged == 0;
  };
  // The solves of a (problem, class, level) block are listed element by
  // element (an element's directions together: they share its data), or,
  // on a handle with shared local matrices, direction by direction
  // (consecutive slots then read the same class matrix).
  const bool dir_major = h->n_cls > 0;
  // The row-per-lane level kernel reads the problem of a wave from its first
  // slot.  With several problems in one launch, each problem's solves start
  // on a whole wave, the gap filled with entries that solve nothing (element
  // -1).  A wave holds 64 / slot solves, the slot being (p+1)^2 lanes rounded
  // up to 4, 8, 16 or 32.
  const bool pad_waves = n_probs > 1;
  auto row_level_kernel = [](int mode) {
    return mode == 0 || mode == 1 || mode == 2 || mode == 6;  // k_sweep_level, not the row-set LU
  };
  auto solves_per_wave = [](int p) {
    const int n = (p + 1) * (p + 1);
    return 64 / (n <= 4 ? 4 : n <= 8 ? 8 : n <= 16 ? 16 : 32);
  };
  size_t n_pad = 0;
  // per level and variant, two level-synchronous launches: the problems the
  // persistent schedule covers, then the others
  for (int L = 0; L < max_levels; ++L)
    for (auto &var : variants)
      for (int pass = 0; pass < 2; ++pass) {
      const bool pass_flow = pass == 0;
      const int off = (int)solves.size();
      for (int k = 0; k < n_probs; ++k) {
        const auto &pl = h->plans[k];
        if (!in_level_variant(pl, var) || L >= pl.n_levels) continue;
        if (flow_ok(pl, var) != pass_flow) continue;
        if (pad_waves && row_level_kernel(var.mode))
          while ((solves.size() - off) % solves_per_wave(var.p) != 0) {
            solves.push_back(make_int2(-1, k << 16));
            ++n_pad;
          }
        for (int g = 0; g < pl.n_groups; ++g) {
          const int *lo = &pl.level_off[(size_t)g * (pl.n_levels + 1)];
          const int32_t *ord = &pl.order[(size_t)g * pl.ne];
          const int b0 = (int)solves.size();
          if (dir_major) {
            for (int d : dirs_of[k][g])
              for (int t = lo[L]; t < lo[L + 1]; ++t) solves.push_back(make_int2(ord[t], d | (k << 16)));
          } else {
            for (int t = lo[L]; t < lo[L + 1]; ++t)
              for (int d : dirs_of[k][g]) solves.push_back(make_int2(ord[t], d | (k << 16)));
          }
          const int b1 = (int)solves.size();
          if (flow_ok(pl, var) && b1 > b0) {
            const int blk = blk_first[k] + g * pl.n_levels + L;
            const int ts = solves_per_round(var.mode, pl.n) * kFlowRounds;
            auto &tl = flow_tasks[var];
            blk_solve0[blk] = b0;
            blk_task0[blk] = (int)tl.size();
            for (int x = b0; x < b1; x += ts) {
              tl.push_back(make_int2(x, std::min(ts, b1 - x)));
              flow_task_blk[var].push_back(blk);
            }
          }
        }
      }
      const int cnt = (int)solves.size() - off;
      if (cnt > 0) {
        const TableSet &ts = h->tables[std::make_pair(var.p, var.nq)];
        h->levels[L].push_back({var, off, cnt, affine_tables(var.mode) ? ts.dev_A : ts.dev_T, pass_flow});
      }
      }
  if (solves.size() != total + n_pad) return set_err(h, VEF_ERR_INVALID, "internal: solve list size mismatch");
  if (solves.size() > (size_t)0x7fffffff) return set_err(h, VEF_ERR_INVALID, "too many element-direction pairs");
  he = upload(h, &h->d_solves, solves.data(), solves.size());
  if (he != hipSuccess) return hip_fail(h, he, "upload solve lists");
  {
    // descriptors of the level lists' solves, so that a level launch reads
    // one record per solve instead of the list and then the element's masks
    // and neighbours: flags = inflow faces | neighbour faces << 4 |
    // pivoting needed << 12 | boundary faces << 16; then the solve's class
    // of shared local matrices
    std::vector<int4> desc(2 * solves.size());
    for (size_t i = 0; i < solves.size(); ++i) {
      const int e = solves[i].x, d = solves[i].y & 0xffff, k = solves[i].y >> 16;
      if (e < 0) {  // padding: solves nothing
        desc[2 * i] = make_int4(-1, solves[i].y, 0, 0);
        desc[2 * i + 1] = make_int4(-1, -1, -1, -1);
        continue;
      }
      const auto &pl = h->plans[k];
      const unsigned mk = pl.mask[(size_t)d * pl.ne + e];
      int fl = (int)((mk & 15u) | ((mk >> 7) << 12));
      int nb[4];
      for (int f = 0; f < 4; ++f) {
        nb[f] = pl.nbr[4 * (size_t)e + f];
        fl |= ((int)pl.nbr_face[4 * (size_t)e + f] & 3) << (4 + 2 * f);
        fl |= (nb[f] < 0 ? 1 : 0) << (16 + f);
      }
      // fourth field: the solve's class of shared local matrices, or the
      // entry of its pivot order (element matrices, uncertified solves)
      int w = h->n_cls > 0 ? shared.of(pl, e, d) : 0;
      if (mk & 0x80u) {
        const auto &ix = piv_index[k];
        const auto it = ix.find((long long)d * pl.ne + e);
        if (it != ix.end()) w = it->second;
      }
      desc[2 * i] = make_int4(e, solves[i].y, fl, w);
      desc[2 * i + 1] = make_int4(nb[0], nb[1], nb[2], nb[3]);
    }
    he = upload(h, &h->d_solve_desc, desc.data(), desc.size());
    if (he != hipSuccess) return hip_fail(h, he, "upload solve descriptors");
  }
  if (!flow_tasks.empty()) {
    // predecessors of a task: for each of its solves (e, d) and each inflow
    // face of e with an upwind element u, the task holding the solve (u, d)
    // (same class, so the same position of d in the class's direction list)
    std::vector<std::vector<int>> rank(n_probs);  // [class][element]: position within its level
    for (int k = 0; k < n_probs; ++k) {
      const auto &pl = h->plans[k];
      rank[k].assign((size_t)pl.n_groups * pl.ne, 0);
      for (int g = 0; g < pl.n_groups; ++g) {
        const int *lo = &pl.level_off[(size_t)g * (pl.n_levels + 1)];
        const int32_t *ord = &pl.order[(size_t)g * pl.ne];
        for (int L = 0; L < pl.n_levels; ++L)
          for (int t = lo[L]; t < lo[L + 1]; ++t) rank[k][(size_t)g * pl.ne + ord[t]] = t - lo[L];
      }
    }
    std::vector<int2> ft;
    std::vector<int> pptr(1, 0), pidx;
    for (auto &kv : flow_tasks) {
      const Variant &var = kv.first;
      const int base = (int)ft.size();
      const TableSet &ts = h->tables[std::make_pair(var.p, var.nq)];
      h->flow.push_back({var, base, (int)kv.second.size(), affine_tables(var.mode) ? ts.dev_A : ts.dev_T});
      const int tsz = solves_per_round(var.mode, (var.p + 1) * (var.p + 1)) * kFlowRounds;
      const auto &blks = flow_task_blk[var];
      std::vector<int> pre;
      for (size_t i = 0; i < kv.second.size(); ++i) {
        const int2 tk = kv.second[i];
        const int blk = blks[i];
        const int k = (int)(std::upper_bound(blk_first.begin(), blk_first.end(), blk) - blk_first.begin()) - 1;
        const auto &pl = h->plans[k];
        const int g = (blk - blk_first[k]) / pl.n_levels;
        const int nd_g = (int)dirs_of[k][g].size();
        const int *lo_g = &pl.level_off[(size_t)g * (pl.n_levels + 1)];
        const int Lb = (blk - blk_first[k]) % pl.n_levels;
        const int wb = lo_g[Lb + 1] - lo_g[Lb];  // elements of the task's level
        pre.clear();
        for (int x = tk.x; x < tk.x + tk.y; ++x) {
          const int e = solves[x].x, d = solves[x].y & 0xffff;
          const int di = dir_major ? (x - blk_solve0[blk]) / wb : (x - blk_solve0[blk]) % nd_g;
          const unsigned inflow = pl.mask[(size_t)d * pl.ne + e] & 15u;
          for (int f = 0; f < 4; ++f) {
            const int u = pl.nbr[4 * (size_t)e + f];
            if (!((inflow >> f) & 1u) || u < 0) continue;
            const int Lu = pl.level[(size_t)g * pl.ne + u];
            const int bu = blk_first[k] + g * pl.n_levels + Lu;
            const int ru = rank[k][(size_t)g * pl.ne + u];
            const int pos = dir_major ? di * (lo_g[Lu + 1] - lo_g[Lu]) + ru : ru * nd_g + di;
            const int pt = base + blk_task0[bu] + pos / tsz;
            if (std::find(pre.begin(), pre.end(), pt) == pre.end()) pre.push_back(pt);
          }
        }
        pidx.insert(pidx.end(), pre.begin(), pre.end());
        pptr.push_back((int)pidx.size());
      }
      ft.insert(ft.end(), kv.second.begin(), kv.second.end());
    }
    h->n_flow_tasks = (int)ft.size();
    he = upload(h, &h->d_flow_tasks, ft.data(), ft.size());
    if (he == hipSuccess) he = upload(h, &h->d_pred_ptr, pptr.data(), pptr.size());
    if (he == hipSuccess) he = upload(h, &h->d_pred_idx, pidx.data(), pidx.size());
    if (he == hipSuccess) he = dev_alloc(h, &h->d_flow_flags, (size_t)h->n_flow_tasks + 1);
    if (he == hipSuccess) he = hipMemset(h->d_flow_flags, 0, sizeof(int) * ((size_t)h->n_flow_tasks + 1));
    if (he != hipSuccess) return hip_fail(h, he, "upload persistent task lists");
  }
  // direction-resident tasks: (problem, direction) per variant, one list per kernel choice
  std::vector<int2> tasks;
  for (int pipe = 0; pipe < 2; ++pipe)
    for (auto &var : variants) {
      const int off = (int)tasks.size();
      int width = 1, maxl = 1, gap = 0;
      for (int k = 0; k < n_probs; ++k) {
        const auto &pl = h->plans[k];
        if (!(pl.p == var.p && pl.nq == var.nq && mode_of(pl, VEF_DIR_RESIDENT, pipe != 0, h->fixup) == var.mode)) continue;
        for (int d = 0; d < pl.nd; ++d) tasks.push_back(make_int2(k, d));
        width = std::max(width, pl.max_width);
        maxl = std::max(maxl, pl.n_levels);
        gap = std::max(gap, pl.max_gap);
      }
      const int cnt = (int)tasks.size() - off;
      if (cnt > 0) {
        const TableSet &ts = h->tables[std::make_pair(var.p, var.nq)];
        (pipe ? h->dir_pipe : h->dir_rows)
            .push_back({var, off, cnt, width, maxl, gap, affine_tables(var.mode) ? ts.dev_A : ts.dev_T, ts.dev_T});
      }
    }
  he = upload(h, &h->d_dir_tasks, tasks.data(), tasks.size());
  if (he != hipSuccess) return hip_fail(h, he, "upload direction tasks");
  h->psi_internal.assign(n_probs, nullptr);
  // a problem with lagged couplings keeps its angular flux between runs when
  // the caller passes none: allocated here, zero, so that lagged couplings of
  // the first sweep read zero
  for (int k = 0; k < n_probs; ++k) {
    const auto &pl = h->plans[k];
    if (!pl.n_lagged) continue;
    const size_t bytes = std::max<size_t>((size_t)pl.nd * pl.ne * pl.n * (fp32 ? 4 : 8), 16);
    he = hipMalloc(&h->psi_internal[k], bytes);
    if (he != hipSuccess) {
      h->psi_internal[k] = nullptr;
      return hip_fail(h, he, "allocate angular flux");
    }
    he = hipMemset(h->psi_internal[k], 0, bytes);
    if (he == hipSuccess) he = hipDeviceSynchronize();
    if (he != hipSuccess) return hip_fail(h, he, "clear angular flux");
  }
  h->resid_scratch.assign(n_probs, nullptr);
  h->resid_cap.assign(n_probs, 0);
  return VEF_OK;
}

bool same_io(const vefk::KIO &a, const vefk::KIO &b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

}  // namespace

extern "C" {

int vef_sweep_create(const vef_problem_desc *probs, int n_probs, const vef_options *opt,
                     vef_sweep_t **out) {
  if (!out) return set_err(nullptr, VEF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!probs || n_probs < 1) return set_err(nullptr, VEF_ERR_INVALID, "no problems");
  vef_sweep *h = new (std::nothrow) vef_sweep();
  if (!h) return set_err(nullptr, VEF_ERR_OOM, "host allocation failed");
  int rc;
  try {
    rc = create_impl(probs, n_probs, opt, h);
  } catch (const std::bad_alloc &) {
    rc = set_err(h, VEF_ERR_OOM, "host allocation failed");
  }
  if (rc) {
    g_create_error = h->err;
    free_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return VEF_OK;
}

}  // extern "C"

namespace {

// One run (vef_sweep_run).  no_alloc (vef_sweep_run_static): residuals of
// problems without a caller buffer go to the static array, an internal
// angular flux must already exist, and no timing events are recorded, so that
// the call allocates nothing.
int run_impl(vef_sweep_t *h, const vef_run_args *a, void *stream, bool no_alloc) {
  if (!h) return VEF_ERR_INVALID;
  if (!a || !a->io || a->n_iter < 1) return set_err(h, VEF_ERR_INVALID, "bad run arguments");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int np = (int)h->plans.size();
  const bool fp32 = h->precision == VEF_FP32_LOCAL;
  const size_t esz = fp32 ? sizeof(float) : sizeof(double);
  const bool timing = h->timing && !no_alloc;
  hipError_t he;
  std::vector<vefk::KIO> io(np);
  size_t static_used = 0;
  for (int k = 0; k < np; ++k) {
    const vef_problem_io &u = a->io[k];
    if (!u.mom) return set_err(h, VEF_ERR_INVALID, "mom is NULL for problem " + std::to_string(k));
    if (no_alloc && !u.psi_out && !h->psi_internal[k])
      return set_err(h, VEF_ERR_INVALID, "psi_out is NULL for problem " + std::to_string(k) +
                                             ", which has no internal angular flux yet");
    if (no_alloc && !u.resid) {
      if (static_used + (size_t)a->n_iter > (size_t)VEF_STATIC_RESID_MAX)
        return set_err(h, VEF_ERR_INVALID, "the residuals of problems without a resid buffer need more than "
                                           "VEF_STATIC_RESID_MAX doubles");
      static_used += (size_t)a->n_iter;
    }
  }
  static_used = 0;
  for (int k = 0; k < np; ++k) {
    const vef_problem_io &u = a->io[k];
    const auto &pl = h->plans[k];
    void *psi = u.psi_out;
    if (!psi) {
      if (!h->psi_internal[k]) {
        he = hipMalloc(&h->psi_internal[k], std::max<size_t>((size_t)pl.nd * pl.ne * pl.n * esz, 16));
        if (he != hipSuccess) {
          h->psi_internal[k] = nullptr;
          return hip_fail(h, he, "allocate angular flux");
        }
      }
      psi = h->psi_internal[k];
    }
    double *resid = u.resid;
    if (!resid && no_alloc) {
      resid = h->static_resid + static_used;
      static_used += (size_t)a->n_iter;
    } else if (!resid) {
      if (h->resid_cap[k] < a->n_iter) {
        if (h->resid_scratch[k]) {
          (void)hipDeviceSynchronize();
          (void)hipFree(h->resid_scratch[k]);
          h->resid_scratch[k] = nullptr;
        }
        he = hipMalloc((void **)&h->resid_scratch[k], sizeof(double) * a->n_iter);
        if (he != hipSuccess) return hip_fail(h, he, "allocate residual scratch");
        h->resid_cap[k] = a->n_iter;
      }
      resid = h->resid_scratch[k];
    }
    io[k] = vefk::KIO{u.phi_in, u.q_iso, u.q_dir, u.psi_bc, u.mom, psi, resid};
  }
  bool changed = !h->io_valid;
  for (int k = 0; k < np && !changed; ++k) changed = !same_io(io[k], h->io_last[k]);
  if (changed) {
    // the pinned staging buffer may still feed a previous upload
    he = hipEventSynchronize(h->io_uploaded);
    if (he != hipSuccess) return hip_fail(h, he, "wait for previous upload");
    std::memcpy(h->h_io_pinned, io.data(), sizeof(vefk::KIO) * np);
    he = hipMemcpyAsync(h->d_io, h->h_io_pinned, sizeof(vefk::KIO) * np, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipEventRecord(h->io_uploaded, s);
    if (he != hipSuccess) return hip_fail(h, he, "upload run pointers");
    h->io_last = io;
    h->io_valid = true;
  }
  int *stop = h->d_flags, *iters = h->d_flags + 1, *status = h->d_flags + 2;
  if (!timing) h->timed_iters = 0;
  if (timing) {
    while ((int)h->events.size() < 2 * a->n_iter) {
      hipEvent_t ev;
      he = hipEventCreate(&ev);
      if (he != hipSuccess) return hip_fail(h, he, "create timing event");
      h->events.push_back(ev);
    }
    h->timed_iters = a->n_iter;
    h->timed_launches = 0;
  }
  auto timed = [&](int it) {
    return timing && ((it + 1) % h->timing_stride == 0 || it == a->n_iter - 1);
  };
  he = vefk::launch_run_init(h->d_io, np, a->n_iter, stop, iters, status, s);
  if (he != hipSuccess) return hip_fail(h, he, "launch init");
  const bool persistent = h->schedule == VEF_PERSISTENT;
  // level-synchronous row-set LU launches solve with the class matrices,
  // which every run forms before its first sweep
  const bool use_cls = h->n_cls > 0 && !h->shared_lu && h->schedule == VEF_LEVEL_SYNC;
  if (persistent && !h->flow.empty()) {
    // task flags and the abort flag start from zero in every run
    he = vefk::launch_zero_ints(h->d_flow_flags, h->n_flow_tasks + 1, s);
    if (he != hipSuccess) return hip_fail(h, he, "launch flag reset");
  }
  for (int it = 0; it < a->n_iter; ++it) {
    if (timed(it) && (he = hipEventRecord(h->events[2 * it], s)) != hipSuccess)
      return hip_fail(h, he, "record timing event");
    vefk::SweepLaunch SL{};
    SL.fp32 = fp32;
    SL.probs = h->d_probs;
    SL.io = h->d_io;
    SL.it = it;
    SL.stop = stop;
    SL.status = status;
    SL.block = h->block;
    SL.lds_max = h->lds_max;
    SL.stream = s;
    SL.waves = h->pipeline_waves > 0 ? h->pipeline_waves : 0;
    SL.ring = h->pipeline_ring;
    SL.fixup = h->fixup;
    SL.wait_spins = h->wait_polls;
    SL.n_cu = h->n_cu;
    SL.single = h->h_probs.size() == 1;
    if (use_cls && it == 0) {
      const auto &pl = h->plans[0];
      vefk::ClassInvLaunch C{};
      C.p = pl.p;
      C.nq = pl.nq;
      C.fp32 = fp32;
      C.n_cls = h->n_cls;
      C.rep = h->d_cls_rep;
      C.probs = h->d_probs;
      C.tables = h->tables[std::make_pair(pl.p, pl.nq)].dev_A;
      C.out = h->d_cls_inv;
      C.status = status;
      C.stream = s;
      he = vefk::launch_class_inv(C);
      if (he != hipSuccess) return hip_fail(h, he, "launch class matrices");
      if (timed(it)) h->timed_launches++;
    }
    if (persistent) {
      for (auto &F : h->flow) {
        SL.p = F.v.p;
        SL.nq = F.v.nq;
        SL.mode = launch_mode(h->mat_quadrature, F.v.mode);
        SL.flow = true;
        SL.list = h->d_solves;
        SL.desc = h->d_solve_desc;  // the records of the whole solve list, indexed as the tasks index it
        SL.tasks = h->d_flow_tasks + F.off;
        SL.count = F.cnt;
        SL.pred_ptr = h->d_pred_ptr + F.off;
        SL.pred_idx = h->d_pred_idx;
        SL.flags = h->d_flow_flags;
        SL.own_base = F.off;
        SL.abort_flag = h->d_flow_flags + h->n_flow_tasks;
        SL.n_cu = h->n_cu;
        SL.tables = F.tab;
        he = vefk::launch_sweep_level(SL);
        if (he != hipSuccess) return hip_fail(h, he, "launch persistent sweep");
        if (timed(it)) h->timed_launches++;
      }
      SL.flow = false;
    }
    if (h->schedule == VEF_LEVEL_SYNC || persistent) {
      for (auto &lv : h->levels)
        for (auto &L : lv) {
          if (persistent && L.flow) continue;  // in a persistent launch
          SL.p = L.v.p;
          SL.nq = L.v.nq;
          SL.mode = launch_mode(h->mat_quadrature, L.v.mode);
          SL.shared = use_cls && L.v.mode == 5;
          SL.list = h->d_solves + L.off;
          SL.desc = h->d_solve_desc + 2 * (size_t)L.off;
          SL.count = L.cnt;
          SL.tables = L.tab;
          he = vefk::launch_sweep_level(SL);
          if (he != hipSuccess) return hip_fail(h, he, "launch sweep");
          if (timed(it)) h->timed_launches++;
        }
    } else {
      for (auto &D : (h->pipeline_waves >= 0 ? h->dir_pipe : h->dir_rows)) {
        SL.p = D.v.p;
        SL.nq = D.v.nq;
        SL.mode = launch_mode(h->mat_quadrature, D.v.mode);
        SL.list = h->d_dir_tasks + D.off;
        SL.count = D.cnt;
        SL.width = D.width;
        SL.max_levels = D.max_levels;
        SL.max_gap = D.max_gap;
        SL.tables = D.tab;
        SL.tables_g = D.tab_g;
        he = vefk::launch_sweep_dir(SL);
        if (he != hipSuccess) return hip_fail(h, he, "launch sweep");
        if (timed(it)) h->timed_launches++;
      }
    }
    if (timed(it) && (he = hipEventRecord(h->events[2 * it + 1], s)) != hipSuccess)
      return hip_fail(h, he, "record timing event");
    for (int k = 0; k < np; ++k) {
      const auto &pl = h->plans[k];
      he = vefk::launch_moments(fp32, h->d_probs, h->d_io, k, pl.ne * pl.n, pl.nd, it, stop, s);
      if (he != hipSuccess) return hip_fail(h, he, "launch moments");
    }
    // the stop test needs a tolerance; without one only the count of sweeps
    // is recorded, after the last
    if (a->tol > 0.0 || it == a->n_iter - 1) {
      he = vefk::launch_finalize(h->d_io, np, it, a->tol, stop, iters, a->iters_done, s);
      if (he != hipSuccess) return hip_fail(h, he, "launch finalize");
    }
  }
  // Boundary sums for E_b and J_in, once, from the angular flux of the last
  // sweep performed (later sweeps skipped by the tolerance test leave it).
  for (int k = 0; k < np; ++k) {
    const auto &pl = h->plans[k];
    he = vefk::launch_boundary(fp32, h->d_probs, h->d_io, k, pl.nbf, pl.nq, pl.p, nullptr, s);
    if (he != hipSuccess) return hip_fail(h, he, "launch boundary sums");
  }
  h->last_stream = s;
  return VEF_OK;
}

}  // namespace

extern "C" {

int vef_sweep_run(vef_sweep_t *h, const vef_run_args *a, void *stream) { return run_impl(h, a, stream, false); }

int vef_sweep_run_static(vef_sweep_t *h, const vef_run_args *a, void *stream) {
  return run_impl(h, a, stream, true);
}

int vef_moments(vef_sweep_t *h, const vef_moment_io *io, void *stream) {
  if (!h) return VEF_ERR_INVALID;
  if (!io) return set_err(h, VEF_ERR_INVALID, "io is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int np = (int)h->plans.size();
  std::vector<vefk::KMomIO> m(np);
  for (int k = 0; k < np; ++k) {
    const vef_moment_io &u = io[k];
    if (u.E && !u.mom) return set_err(h, VEF_ERR_INVALID, "E requested without mom");
    m[k] = vefk::KMomIO{u.mom, u.q_iso, u.q_dir, u.psi_bc, u.E, u.Eb, u.Jin, u.Q0, u.Q1, u.n_nonpos};
  }
  // same pointers as the last call: kernel launches only (capturable)
  bool changed = !h->mio_valid;
  for (int k = 0; k < np && !changed; ++k)
    changed = std::memcmp(&m[k], &h->mio_last[k], sizeof(vefk::KMomIO)) != 0;
  hipError_t he = hipSuccess;
  if (changed) {
    he = hipEventSynchronize(h->mio_uploaded);
    if (he != hipSuccess) return hip_fail(h, he, "wait for previous closure upload");
    std::memcpy(h->h_mio_pinned, m.data(), sizeof(vefk::KMomIO) * np);
    he = hipMemcpyAsync(h->d_mio, h->h_mio_pinned, sizeof(vefk::KMomIO) * np, hipMemcpyHostToDevice, s);
    if (he == hipSuccess) he = hipEventRecord(h->mio_uploaded, s);
    if (he != hipSuccess) return hip_fail(h, he, "upload closure pointers");
    h->mio_last = m;
    h->mio_valid = true;
  }
  he = vefk::launch_zero_nonpos(h->d_mio, np, s);
  if (he != hipSuccess) return hip_fail(h, he, "upload closure pointers");
  for (int k = 0; k < np; ++k) {
    const auto &pl = h->plans[k];
    he = vefk::launch_closures(h->d_probs, h->d_mio, k, pl.ne, pl.Q, pl.n, pl.nbf, pl.nq, s);
    if (he != hipSuccess) return hip_fail(h, he, "launch closures");
  }
  h->last_stream = s;
  return VEF_OK;
}

int vef_sweep_destroy(vef_sweep_t *h) {
  if (!h) return VEF_OK;
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
  return VEF_OK;
}

int vef_plan_query(const vef_problem_desc *prob, const vef_options *opt, vef_info *info) {
  if (!prob) return set_err(nullptr, VEF_ERR_INVALID, "prob is NULL");
  const int cycles = opt ? opt->cycles : VEF_CYCLES_REJECT;
  if (cycles != VEF_CYCLES_REJECT && cycles != VEF_CYCLES_LAG)
    return set_err(nullptr, VEF_ERR_INVALID, "cycles must be VEF_CYCLES_REJECT or VEF_CYCLES_LAG");
  const int upwind = opt ? opt->upwind : VEF_UPWIND_FACE;
  if (upwind != VEF_UPWIND_FACE && upwind != VEF_UPWIND_POINT)
    return set_err(nullptr, VEF_ERR_INVALID, "unknown upwind rule");
  vefplan::ProblemPlan pl;
  std::string e;
  int rc;
  try {
    rc = vefplan::build_problem_plan(*prob, cycles == VEF_CYCLES_LAG, upwind == VEF_UPWIND_POINT, pl, e);
  } catch (const std::bad_alloc &) {
    return set_err(nullptr, VEF_ERR_OOM, "host allocation failed");
  }
  if (rc) return set_err(nullptr, rc, e);
  if (info) {
    info->n = pl.n;
    info->nq = pl.nq;
    info->Q = pl.Q;
    info->n_bf = pl.nbf;
    info->n_levels = pl.n_levels;
    info->n_groups = pl.n_groups;
    info->pivoting = pl.nopivot ? 0 : 1;
    info->affine = pl.affine ? 1 : 0;
    info->n_solves = (long long)pl.ne * pl.nd;
    info->schedule = VEF_SCHEDULE_AUTO;
    info->kernel = -1;
    info->n_lagged = pl.n_lagged;
    info->n_pivoting = pl.nopivot ? 0 : pl.n_pivoting;
    info->n_classes = 0;
    if ((!opt || opt->shared_matrices == 0) && mode_of(pl, VEF_LEVEL_SYNC) == 5) {
      const bool fp32 = opt && opt->precision == VEF_FP32_LOCAL;
      SharedClasses sc;
      try {
        if (find_shared_classes(pl, class_matrix_entries(pl) * (fp32 ? sizeof(float) : sizeof(double)), sc))
          info->n_classes = sc.n_cls;
      } catch (const std::bad_alloc &) {
        return set_err(nullptr, VEF_ERR_OOM, "host allocation failed");
      }
    }
  }
  return VEF_OK;
}

int vef_problem_info(const vef_sweep_t *h, int k, vef_info *info) {
  if (!h || !info || k < 0 || k >= (int)h->plans.size()) return VEF_ERR_INVALID;
  const auto &pl = h->plans[k];
  info->n = pl.n;
  info->nq = pl.nq;
  info->Q = pl.Q;
  info->n_bf = pl.nbf;
  info->n_levels = pl.n_levels;
  info->n_groups = pl.n_groups;
  info->pivoting = pl.nopivot ? 0 : 1;
  info->affine = pl.affine ? 1 : 0;
  info->n_solves = (long long)pl.ne * pl.nd;
  info->schedule = h->schedule;
  info->kernel = launch_mode(h->mat_quadrature, mode_of(pl, h->schedule, h->pipeline_waves >= 0, h->fixup));
  if (info->kernel == VEF_KERNEL_AFFINE_LU && h->n_cls > 0 && !h->shared_lu && h->schedule == VEF_LEVEL_SYNC)
    info->kernel = VEF_KERNEL_AFFINE_SHARED;
  info->n_lagged = pl.n_lagged;
  info->n_pivoting = pl.nopivot ? 0 : pl.n_pivoting;
  info->n_classes = h->n_cls;
  return VEF_OK;
}

static int hrt_setup(vef_sweep_t *h, int k) {
  const auto &pl = h->plans[k];
  hipError_t he;
  // set-up on first use (not in a captured region): affine geometry in
  // double precision and the tables of (p, nq)
  if (h->hrt_geo.size() != h->plans.size()) h->hrt_geo.assign(h->plans.size(), nullptr);
  if (!h->hrt_geo[k]) {
    std::vector<double> g((size_t)pl.ne * 13);
    for (int e = 0; e < pl.ne; ++e)
      for (int i = 0; i < 13; ++i) g[(size_t)e * 13 + i] = pl.geo_a[(size_t)e * 16 + i];
    double *d = nullptr;
    he = hipMalloc(&d, g.size() * sizeof(double));
    if (he == hipSuccess) he = hipMemcpy(d, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      if (d) (void)hipFree(d);
      return hip_fail(h, he, "upload HRT geometry");
    }
    h->hrt_geo[k] = d;
  }
  const auto key = std::make_pair(pl.p, pl.nq);
  if (!h->hrt_tab.count(key)) {
    std::vector<double> blob;
    if (vefplan::build_hrt_tables(pl.p, pl.nq, blob)) return set_err(h, VEF_ERR_INVALID, "HRT tables");
    double *d = nullptr;
    he = hipMalloc(&d, blob.size() * sizeof(double));
    if (he == hipSuccess) he = hipMemcpy(d, blob.data(), blob.size() * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      if (d) (void)hipFree(d);
      return hip_fail(h, he, "upload HRT tables");
    }
    h->hrt_tab[key] = d;
  }
  return VEF_OK;
}

int vef_hrt_local_inverse(vef_sweep_t *h, int k, const double *mom, const double *Eb, double *inv,
                          void *stream) {
  if (!h) return VEF_ERR_INVALID;
  if (k < 0 || k >= (int)h->plans.size()) return set_err(h, VEF_ERR_INVALID, "problem index out of range");
  if (!mom || !inv) return set_err(h, VEF_ERR_INVALID, "mom and inv are required");
  const auto &pl = h->plans[k];
  if (!pl.affine) return set_err(h, VEF_ERR_INVALID, "HRT local blocks need affine elements");
  vefplan::HrtSizes z;
  if (vefplan::hrt_sizes(pl.p, pl.nq, z))
    return set_err(h, VEF_ERR_INVALID, "HRT local blocks need p in 1..3 and nq = p + 2 or p + 3");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t he;
  const int rs = hrt_setup(h, k);
  if (rs != VEF_OK) return rs;
  const auto key = std::make_pair(pl.p, pl.nq);
  vefk::HrtLaunch L{pl.p, pl.nq, pl.ne, h->hrt_tab[key], h->hrt_geo[k], h->h_probs[k].sig, h->h_probs[k].nbr,
                    mom, Eb, inv, s};
  he = vefk::launch_hrt_inverse(L);
  if (he != hipSuccess) return hip_fail(h, he, "launch HRT local inverse");
  h->last_stream = s;
  return VEF_OK;
}

int vef_hrt_reduce(vef_sweep_t *h, int k, const double *mom, const double *Eb, const double *Jin,
                   const double *Q0, const double *Q1, const double *inv, double *hloc, double *rloc,
                   double *sol0, double *resp, void *stream) {
  if (!h) return VEF_ERR_INVALID;
  if (k < 0 || k >= (int)h->plans.size()) return set_err(h, VEF_ERR_INVALID, "problem index out of range");
  if (!mom || !Jin || !Q0 || !Q1 || !inv || !hloc || !rloc || !sol0 || !resp)
    return set_err(h, VEF_ERR_INVALID, "mom, Jin, Q0, Q1, inv and the outputs are required");
  const auto &pl = h->plans[k];
  if (!pl.affine) return set_err(h, VEF_ERR_INVALID, "HRT local blocks need affine elements");
  vefplan::HrtSizes z;
  if (vefplan::hrt_sizes(pl.p, pl.nq, z))
    return set_err(h, VEF_ERR_INVALID, "HRT local blocks need p in 1..3 and nq = p + 2 or p + 3");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rs = hrt_setup(h, k);
  if (rs != VEF_OK) return rs;
  const auto key = std::make_pair(pl.p, pl.nq);
  vefk::HrtReduceLaunch L{pl.p, pl.nq, pl.ne, h->hrt_tab[key], h->hrt_geo[k], h->h_probs[k].nbr,
                          h->h_probs[k].nbr_face, mom, Eb, Jin, Q0, Q1, inv, hloc, rloc, sol0, resp, s};
  const hipError_t he = vefk::launch_hrt_reduce(L);
  if (he != hipSuccess) return hip_fail(h, he, "launch HRT reduction");
  h->last_stream = s;
  return VEF_OK;
}

int vef_boundary_faces(const vef_sweep_t *h, int k, int32_t *out) {
  if (!h || !out || k < 0 || k >= (int)h->plans.size()) return VEF_ERR_INVALID;
  const auto &pl = h->plans[k];
  for (int b = 0; b < pl.nbf; ++b) {
    out[2 * b] = pl.bf_ef[b] >> 2;
    out[2 * b + 1] = pl.bf_ef[b] & 3;
  }
  return VEF_OK;
}

int vef_sweep_autotune(vef_sweep_t *h, const vef_run_args *a, void *stream, int reps, vef_tune_result *out) {
  if (!h) return VEF_ERR_INVALID;
  if (!a || reps < 1 || reps > 1000) return set_err(h, VEF_ERR_INVALID, "bad autotune arguments (reps 1..1000)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  struct Cand {
    int schedule, waves, block;
    bool quad;  // problems with element matrices take the quadrature kernel
    bool lu;    // problems with shared local matrices take the row-set LU
    bool operator==(const Cand &o) const {
      return schedule == o.schedule && waves == o.waves && block == o.block && quad == o.quad && lu == o.lu;
    }
  };
  const Cand before{h->schedule, h->pipeline_waves, h->block, h->mat_quadrature, h->shared_lu};
  bool any_pipe = false, any_mat = false;
  for (auto &pl : h->plans) {
    const int md = mode_of(pl, VEF_DIR_RESIDENT, true, h->fixup);
    any_pipe |= md == 3 || md == 4;
    any_mat |= pl.elem_mat;
  }
  std::vector<Cand> cands{before};
  auto add = [&](Cand c) {
    for (auto &x : cands)
      if (x == c) return;
    cands.push_back(c);
  };
  for (bool quad : {false, true}) {
    // the element-matrix kernel against quadrature assembly (matrix cores
    // against the vector units) where some problem has both
    if (quad && !any_mat) continue;
    // class matrices against the row-set LU (level-synchronous only)
    for (bool lu : {false, true}) {
      if (lu && h->n_cls == 0) continue;
      add({VEF_LEVEL_SYNC, before.waves, 256, quad, lu});
      add({VEF_LEVEL_SYNC, before.waves, 128, quad, lu});
    }
    add({VEF_DIR_RESIDENT, -1, before.block, quad, before.lu});
    if (!h->flow.empty()) add({VEF_PERSISTENT, before.waves, 256, quad, before.lu});
  }
  if (any_pipe)
    for (int w : {8, 6, 4}) add({VEF_DIR_RESIDENT, w, before.block, before.quad, before.lu});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(h, he, "create tuning events");
  }
  auto finish = [&](int rc, const Cand &c) {
    h->schedule = c.schedule;
    h->pipeline_waves = c.waves;
    h->block = c.block;
    h->mat_quadrature = c.quad;
    h->shared_lu = c.lu;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
  };
  double best = 1e300, before_ms = -1.0;
  Cand bestc = before;
  for (const Cand &c : cands) {
    h->schedule = c.schedule;
    h->pipeline_waves = c.waves;
    h->block = c.block;
    h->mat_quadrature = c.quad;
    h->shared_lu = c.lu;
    int rc = vef_sweep_run(h, a, stream);  // warm-up (uploads, first-touch)
    if (rc == VEF_OK && (he = hipEventRecord(e0, s)) != hipSuccess) rc = hip_fail(h, he, "record tuning event");
    for (int r = 0; r < reps && rc == VEF_OK; ++r) rc = vef_sweep_run(h, a, stream);
    if (rc == VEF_OK && (he = hipEventRecord(e1, s)) != hipSuccess) rc = hip_fail(h, he, "record tuning event");
    if (rc == VEF_OK && (he = hipEventSynchronize(e1)) != hipSuccess) rc = hip_fail(h, he, "wait for tuning run");
    if (rc == VEF_OK) rc = vef_sweep_check(h);
    if (rc != VEF_OK) return finish(rc, before);
    float ms = 0.f;
    if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return finish(hip_fail(h, he, "read tuning events"), before);
    const double per = (double)ms / reps;
    if (c == before) before_ms = per;
    if (per < best) {
      best = per;
      bestc = c;
    }
  }
  // timing noise is a few tenths of a percent: keep the configuration the
  // handle had unless another is clearly faster
  if (before_ms >= 0.0 && best * 1.02 > before_ms) {
    bestc = before;
    best = before_ms;
  }
  if (out) {
    out->schedule = bestc.schedule;
    out->pipeline_waves = bestc.waves;
    out->block = bestc.block;
    out->elem_matrices = any_mat ? (bestc.quad ? 0 : 1) : -1;
    out->shared_matrices = h->n_cls > 0 ? (bestc.lu || bestc.schedule != VEF_LEVEL_SYNC ? 0 : 1) : -1;
    out->n_candidates = (int)cands.size();
    out->best_ms = best;
    out->before_ms = before_ms;
  }
  return finish(VEF_OK, bestc);
}

int vef_sweep_check(vef_sweep_t *h) {
  if (!h) return VEF_ERR_INVALID;
  hipError_t he = hipStreamSynchronize(h->last_stream);
  if (he != hipSuccess) return hip_fail(h, he, "stream synchronize");
  int flags[4];
  he = hipMemcpy(flags, h->d_flags, sizeof(flags), hipMemcpyDeviceToHost);
  if (he != hipSuccess) return hip_fail(h, he, "read status");
  if (flags[2] & 2) return set_err(h, VEF_ERR_TIMEOUT, "a pipelined sweep wait exceeded its bound");
  if (flags[2] & 4) return set_err(h, VEF_ERR_INVALID, "internal: a level-synchronous wave held two problems");
  if (flags[2]) return set_err(h, VEF_ERR_INVALID, "non-finite unknown (singular local system)");
  return VEF_OK;
}

int vef_sweep_timing(vef_sweep_t *h, double *sweep_ms, int *n_launches) {
  if (!h) return VEF_ERR_INVALID;
  if (!h->timing) return set_err(h, VEF_ERR_INVALID, "handle was created without timing");
  hipError_t he = hipStreamSynchronize(h->last_stream);
  if (he != hipSuccess) return hip_fail(h, he, "stream synchronize");
  double tot = 0.0;
  for (int it = 0; it < h->timed_iters; ++it) {
    if ((it + 1) % h->timing_stride != 0 && it != h->timed_iters - 1) continue;
    float ms = 0.0f;
    he = hipEventElapsedTime(&ms, h->events[2 * it], h->events[2 * it + 1]);
    if (he != hipSuccess) return hip_fail(h, he, "event elapsed time");
    tot += ms;
  }
  if (sweep_ms) *sweep_ms = tot;
  if (n_launches) *n_launches = h->timed_launches;
  return VEF_OK;
}

const char *vef_last_error(const vef_sweep_t *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

const char *vef_status_string(int status) {
  switch (status) {
    case VEF_OK: return "ok";
    case VEF_ERR_INVALID: return "invalid argument";
    case VEF_ERR_CYCLE: return "cyclic upwind graph";
    case VEF_ERR_JACOBIAN: return "non-positive Jacobian";
    case VEF_ERR_HIP: return "HIP runtime error";
    case VEF_ERR_OOM: return "out of memory";
    case VEF_ERR_TIMEOUT: return "device wait timed out";
    default: return "unknown status";
  }
}

}  // extern "C"

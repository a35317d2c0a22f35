// HIP kernels for gfx950: DG S_N sweep (level-synchronous and
// direction-resident schedules), angular-moment and residual reduction,
// boundary sums and VEF closures.
//
// Sweep work mapping: a "slot" of SLOT lanes (the power of two >= n = (p+1)^2,
// aligned inside one 64-wide wavefront) owns one element-direction solve;
// lane r owns row r (test function r) of the local system.  One solve:
//   1. inputs: the lanes of the slot load the element's geometry factors
//      (w J and w adj(F) at volume points, w n ds at face points), the nodal
//      source coefficients and the direction-dependent source, a few values
//      per lane, all loads independent (the direction-resident schedule
//      issues them one solve ahead);
//   2. staging: those values go to the slot's private LDS area and the
//      source is evaluated at the volume points (wave-local, no work-group
//      barrier);
//   3. assembly: each lane builds its row by quadrature from the LDS data and
//      the basis tables (staged in LDS once per work-group); inflow traces
//      come from the upwind element's face nodes (Gauss-Lobatto nodes include
//      the element boundary, so a face trace is the p+1 face-node values, read
//      in reversed order because the two sides run the shared face in
//      opposite senses);
//   4. solve: Gauss-Jordan elimination with normalised pivot rows across the
//      slot's lanes, so that each lane ends with one unknown.  With partial
//      pivoting the pivot lane is one unsigned max of packed (magnitude, lane)
//      keys by DPP lane moves and the pivot row goes through the slot's LDS
//      area; without pivoting (used only when every face of the mesh is
//      straight and sigma_t > 0, so that the local matrix has a positive
//      definite symmetric part) lane k broadcasts row k by a DPP row
//      broadcast or an LDS swizzle, with no LDS round trip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace vefk {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

template <int P, int NQ>
struct Shape {
  static constexpr int P1 = P + 1;
  static constexpr int N = P1 * P1;
  static constexpr int Q = NQ * NQ;
  static constexpr int SLOT = N <= 4 ? 4 : (N <= 8 ? 8 : (N <= 16 ? 16 : 32));
  static constexpr int SPW = 64 / SLOT;
  // per-lane shares of the element inputs
  static constexpr int GV = (5 * Q + SLOT - 1) / SLOT;
  static constexpr int GF = (8 * NQ + SLOT - 1) / SLOT;
  static constexpr int QD = (Q + SLOT - 1) / SLOT;
  // LDS: tables, then one area per slot
  static constexpr int TAB = 3 * Q * N + NQ * P1;
  static constexpr int OFF_GEO = 0;                 // [Q][5]
  static constexpr int OFF_GF = OFF_GEO + 5 * Q;    // [4][NQ][2]
  static constexpr int OFF_SRC = OFF_GF + 8 * NQ;   // [Q] source at volume points
  static constexpr int OFF_S = OFF_SRC + Q;         // [N] nodal source coefficients
  static constexpr int OFF_PIV = ((OFF_S + N + 1) / 2) * 2;  // [N + 1] pivot row + rhs
  static constexpr int SLOT_AREA = ((OFF_PIV + N + 1 + 1) / 2) * 2;
  // volume loop fully unrolled for the small elements
  static constexpr int QU = P <= 2 ? Q : 1;
};

template <typename T>
__host__ __device__ constexpr size_t lds_bytes(int tab, int slot_area, int slots, int extra_ints) {
  return sizeof(T) * ((size_t)tab + (size_t)slot_area * slots) + sizeof(int) * (size_t)extra_ints;
}

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

// DPP lane moves (whole-wave, all lanes active)
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(dpp_mov<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = dpp_mov<CTRL>(__double2loint(v));
  const int hi = dpp_mov<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// LDS-crossbar swizzle with an immediate bit-mask pattern (32-lane groups)
template <int PAT>
__device__ __forceinline__ int swz(int v) {
  return __builtin_amdgcn_ds_swizzle(v, PAT);
}
template <int PAT>
__device__ __forceinline__ float swz(float v) {
  return __int_as_float(swz<PAT>(__float_as_int(v)));
}
template <int PAT>
__device__ __forceinline__ double swz(double v) {
  const int lo = swz<PAT>(__double2loint(v));
  const int hi = swz<PAT>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Value of lane K of the caller's slot.  16-lane slots are DPP rows
// (row_newbcast:K); other sizes use the swizzle "and/or" mode, which keeps
// the slot bits of the lane id and forces the low bits to K.
template <int SLOT, int K, typename T>
__device__ __forceinline__ T slot_bcast(T v) {
  if constexpr (SLOT == 16) {
    return dpp_mov<0x150 + K>(v);
  } else {
    constexpr int AND = (~(SLOT - 1)) & 0x1F;
    return swz<AND | (K << 5)>(v);
  }
}

// Pivot lane of a slot: each lane offers a key made of its |a_k| rounded
// down to float with the low five mantissa bits replaced by (31 - lane in
// slot); lanes that may not pivot offer 0.  For non-negative floats the bit
// pattern orders like an unsigned integer, so one unsigned max over the slot
// picks the largest magnitude and, among equal keys, the lowest lane.
// quad_perm [1,0,3,2] and [2,3,0,1] pair lanes inside quads, row_half_mirror
// pairs the two quads of an 8-lane group, row_mirror the two halves of a
// 16-lane row; 32-lane slots finish with one cross-row exchange.
template <int SLOT>
__device__ __forceinline__ int slot_pivot(float mag, bool cand, int r) {
  unsigned key = cand ? ((__float_as_uint(mag) & ~31u) | (31u - (unsigned)r)) : 0u;
  key = max(key, (unsigned)dpp_mov<0xB1>((int)key));
  key = max(key, (unsigned)dpp_mov<0x4E>((int)key));
  if constexpr (SLOT >= 8) key = max(key, (unsigned)dpp_mov<0x141>((int)key));
  if constexpr (SLOT >= 16) key = max(key, (unsigned)dpp_mov<0x140>((int)key));
  if constexpr (SLOT >= 32) key = max(key, (unsigned)__shfl_xor((int)key, 16, 32));
  return 31 - (int)(key & 31u);
}

// 1/x from the hardware reciprocal refined by Newton steps (two in double,
// one in float: each step squares the relative error).
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) {
  float y = __builtin_amdgcn_rcpf(x);
  return fmaf(y, fmaf(-x, y, 1.0f), y);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Step K of the pivot-free Gauss-Jordan elimination: lane K's row is the
// pivot row; every lane subtracts l times it, where the pivot lane's own l
// turns its row into the row divided by its pivot.
template <int SLOT, int N, int K, typename T>
__device__ __forceinline__ void gj_nopivot(T (&A)[N], T &rhs, int r) {
  if constexpr (K < N) {
    const T pk = slot_bcast<SLOT, K>(A[K]);
    const T inv = recip(pk);
    const T l = (r == K) ? (A[K] - T(1)) * inv : A[K] * inv;
#pragma unroll
    for (int j = K + 1; j < N; ++j) A[j] -= l * slot_bcast<SLOT, K>(A[j]);
    rhs -= l * slot_bcast<SLOT, K>(rhs);
    gj_nopivot<SLOT, N, K + 1, T>(A, rhs, r);
  }
}

// Step K with partial pivoting; the pivot row travels through LDS.
template <int SLOT, int N, int K, typename T>
__device__ __forceinline__ void gj_pivot(T (&A)[N], T &rhs, int r, bool &active, int &my_k, T *pv) {
  if constexpr (K < N) {
    const int pl = slot_pivot<SLOT>(static_cast<float>(fabs(A[K])), active, r);
    if (r == pl) {
#pragma unroll
      for (int j = K; j < N; ++j) pv[j] = A[j];
      pv[N] = rhs;
      active = false;
      my_k = K;
    }
    wave_sync_lds();
    const T inv = recip(pv[K]);
    const T l = (r == pl) ? (A[K] - T(1)) * inv : A[K] * inv;
#pragma unroll
    for (int j = K + 1; j < N; ++j) A[j] -= l * pv[j];
    rhs -= l * pv[N];
    __builtin_amdgcn_wave_barrier();
    gj_pivot<SLOT, N, K + 1, T>(A, rhs, r, active, my_k, pv);
  }
}

// Per-lane inputs of one solve (loaded ahead of the solve).
template <int P, int NQ, typename T>
struct SolveIn {
  using S = Shape<P, NQ>;
  int e, flags;  // flags: bits 0-3 inflow faces, bits 4+2f.. neighbour's local face
  int nb[4];     // neighbour element, or -(boundary face + 1)
  bool valid;
  T g[S::GV];
  T f[S::GF];
  T s;
  T qd[S::QD];
};

template <int P, int NQ, typename T>
__device__ __forceinline__ void load_inputs(SolveIn<P, NQ, T> &in, int d, const KProb &pb,
                                            const KIO &pio, int it, int r) {
  using S = Shape<P, NQ>;
  constexpr int N = S::N, Q = S::Q, SLOT = S::SLOT;
  const int e = in.e;
  if (!in.valid) return;
  const T *gv = static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5;
#pragma unroll
  for (int k = 0; k < S::GV; ++k) {
    const int i = r + k * SLOT;
    in.g[k] = i < 5 * Q ? gv[i] : T(0);
  }
  const T *gf = static_cast<const T *>(pb.geo_f) + (size_t)e * 8 * NQ;
#pragma unroll
  for (int k = 0; k < S::GF; ++k) {
    const int i = r + k * SLOT;
    in.f[k] = i < 8 * NQ ? gf[i] : T(0);
  }
  const double *phi = it == 0 ? pio.phi_in : pio.mom;
  T sv = T(0);
  if (r < N) {
    if (phi) sv = static_cast<T>(pb.sig[2 * e + 1] * kInv4Pi) * static_cast<T>(phi[(size_t)e * N + r]);
    if (pio.q_iso) sv += static_cast<T>(pio.q_iso[(size_t)e * N + r]);
  }
  in.s = sv;
#pragma unroll
  for (int k = 0; k < S::QD; ++k) {
    const int q = r + k * SLOT;
    in.qd[k] = (pio.q_dir && q < Q) ? static_cast<T>(pio.q_dir[((size_t)d * pb.ne + e) * Q + q]) : T(0);
  }
}

// Assemble and solve one element-direction system from prefetched inputs.
// All lanes of the slot must call it; slots with in.valid == false store
// nothing.  Uses only the slot's LDS area (no work-group barrier inside).
template <int P, int NQ, typename T, bool PIVOT>
__device__ __forceinline__ void solve_from(const SolveIn<P, NQ, T> &in, int d, const KProb &pb,
                                           const KIO &pio, T *lds, int r, int slot, int *status) {
  using S = Shape<P, NQ>;
  constexpr int P1 = S::P1, N = S::N, Q = S::Q, SLOT = S::SLOT;
  const T *sV = lds;
  const T *sDx = lds + Q * N;
  const T *sDy = lds + 2 * Q * N;
  const T *sF = lds + 3 * Q * N;
  T *area = lds + S::TAB + (size_t)slot * S::SLOT_AREA;
  const int ne = pb.ne;
  const int e = in.e;
  const bool valid = in.valid;
  const bool row_ok = valid && r < N;
  const int rr = r < N ? r : N - 1;  // table index for padding lanes
  const int a = rr % P1, b = rr / P1;
  const unsigned mask = valid ? (unsigned)in.flags & 15u : 0u;
  const T *psi = static_cast<const T *>(pio.psi);

  // upwind traces: the only loads on the critical path
  T tr[4][P1];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
#pragma unroll
    for (int c = 0; c < P1; ++c) tr[f][c] = T(0);
    if (row_ok && on_face && ((mask >> f) & 1u) && in.nb[f] >= 0) {
      const int f2 = (in.flags >> (4 + 2 * f)) & 3;
      const T *up = psi + ((size_t)d * ne + in.nb[f]) * N;
#pragma unroll
      for (int c = 0; c < P1; ++c) tr[f][c] = up[face_node<P>(f2, P - c)];
    }
  }

  // staging (wave-local)
#pragma unroll
  for (int k = 0; k < S::GV; ++k) {
    const int i = r + k * SLOT;
    if (i < 5 * Q) area[S::OFF_GEO + i] = in.g[k];
  }
#pragma unroll
  for (int k = 0; k < S::GF; ++k) {
    const int i = r + k * SLOT;
    if (i < 8 * NQ) area[S::OFF_GF + i] = in.f[k];
  }
  if (r < N) area[S::OFF_S + r] = in.s;
  wave_sync_lds();
#pragma unroll
  for (int k = 0; k < S::QD; ++k) {
    const int q = r + k * SLOT;
    if (q < Q) {
      T src = in.qd[k];
#pragma unroll
      for (int j = 0; j < N; ++j) src += area[S::OFF_S + j] * sV[q * N + j];
      area[S::OFF_SRC + q] = src;
    }
  }
  wave_sync_lds();

  // assembly of row r
  const T ox = static_cast<T>(pb.omega[2 * d]);
  const T oy = static_cast<T>(pb.omega[2 * d + 1]);
  const T st = static_cast<T>(pb.sig[2 * (valid ? e : 0)]);
  T A[N];
#pragma unroll
  for (int j = 0; j < N; ++j) A[j] = T(0);
  T rhs = T(0);
  const T *g5 = area + S::OFF_GEO;
  const T *srcq = area + S::OFF_SRC;
#pragma unroll S::QU
  for (int q = 0; q < Q; ++q) {
    const T wJ = g5[5 * q], a00 = g5[5 * q + 1], a01 = g5[5 * q + 2], a10 = g5[5 * q + 3], a11 = g5[5 * q + 4];
    const T gx = a00 * ox + a01 * oy;
    const T gy = a10 * ox + a11 * oy;
    const T li = sV[q * N + rr];
    const T c = st * wJ * li - (gx * sDx[q * N + rr] + gy * sDy[q * N + rr]);
    rhs += wJ * li * srcq[q];
#pragma unroll
    for (int j = 0; j < N; ++j) A[j] += c * sV[q * N + j];
  }

  // face terms
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
    const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
    const T *gf = area + S::OFF_GF + f * NQ * 2;
    if (!(row_ok && on_face)) continue;
    if (!((mask >> f) & 1u)) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
        const T t = on * sF[q * P1 + pos];
#pragma unroll
        for (int c = 0; c < P1; ++c) A[face_node<P>(f, c)] += t * sF[q * P1 + c];
      }
    } else if (in.nb[f] >= 0) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        T ph = T(0);
#pragma unroll
        for (int c = 0; c < P1; ++c) ph += tr[f][c] * sF[q * P1 + c];
        const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
        rhs -= on * sF[q * P1 + pos] * ph;
      }
    } else if (pio.psi_bc) {
      const double *bc = pio.psi_bc + ((size_t)d * pb.nbf + (-in.nb[f] - 1)) * NQ;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
        rhs -= on * sF[q * P1 + pos] * static_cast<T>(bc[q]);
      }
    }
  }

  // Gauss-Jordan elimination; lane r ends with unknown my_k in rhs
  int my_k = r;
  if constexpr (PIVOT) {
    bool active = row_ok;
    gj_pivot<SLOT, N, 0, T>(A, rhs, r, active, my_k, area + S::OFF_PIV);
  } else {
    gj_nopivot<SLOT, N, 0, T>(A, rhs, r);
  }
  if (row_ok) {
    T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
    out[my_k] = rhs;
    if (!(rhs == rhs) || rhs - rhs != T(0)) atomicOr(status, 1);  // non-finite unknown
  }
}

// Stage the basis tables of (P, NQ) into LDS.
template <int P, int NQ, typename T>
__device__ __forceinline__ void stage_tables(const T *__restrict__ tables, T *lds) {
  constexpr int TAB = Shape<P, NQ>::TAB;
  for (int i = threadIdx.x; i < TAB; i += blockDim.x) lds[i] = tables[i];
}

// Level-synchronous schedule: one launch per upwind level over the list of
// (element, direction | problem << 16) pairs of that level.
template <int P, int NQ, typename T, bool PIVOT>
__global__ void __launch_bounds__(256)
k_sweep_level(const int2 *__restrict__ solves, int n_solves, const KProb *__restrict__ probs,
              const KIO *__restrict__ io, const T *__restrict__ tables, int it,
              const int *__restrict__ stop, int *__restrict__ status) {
  using S = Shape<P, NQ>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  if (*stop) return;
  stage_tables<P, NQ, T>(tables, lds);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int r = lane & (S::SLOT - 1);
  const int slot = (threadIdx.x >> 6) * S::SPW + lane / S::SLOT;
  const int sid = blockIdx.x * ((blockDim.x >> 6) * S::SPW) + slot;
  SolveIn<P, NQ, T> in;
  in.valid = sid < n_solves;
  int d = 0, prob = 0;
  in.e = 0;
  in.flags = 0;
  if (in.valid) {
    const int2 sv = solves[sid];
    in.e = sv.x;
    d = sv.y & 0xffff;
    prob = sv.y >> 16;
  }
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  if (in.valid) {
    in.flags = pb.mask[(size_t)d * pb.ne + in.e];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      in.nb[f] = pb.nbr[4 * in.e + f];
      in.flags |= ((int)pb.nbr_face[4 * in.e + f] & 3) << (4 + 2 * f);
    }
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) in.nb[f] = -1;
  }
  load_inputs<P, NQ, T>(in, d, pb, pio, it, r);
  solve_from<P, NQ, T, PIVOT>(in, d, pb, pio, lds, r, slot, status);
}

// Largest work-group of the direction-resident schedule for a (P, NQ, T)
// variant, chosen so that the kernel's registers fit without spilling
// (a 1024-thread group leaves 128 VGPRs per lane, 512 leaves 256).
template <int P, int NQ, typename T>
constexpr int dir_block_max() {
  if (sizeof(T) == 8) return 512;
  return (P == 4 && NQ >= 6) ? 512 : 1024;
}

// Direction-resident schedule: work-group b sweeps one (problem, direction)
// pair through all upwind levels of its direction class.  The elements of a
// level are solved in rounds of (blockDim / SLOT) slots; each slot loads the
// inputs of its next solve before computing the current one, and a
// work-group barrier separates consecutive levels (upwind values were
// written by this work-group, so work-group scope visibility suffices).
// Element descriptors (id, inflow mask, neighbours) come packed in level
// order per direction class; the level offsets sit in LDS.
template <int P, int NQ, typename T, bool PIVOT>
__global__ void __launch_bounds__((dir_block_max<P, NQ, T>()))
k_sweep_dir(const int2 *__restrict__ tasks, const KProb *__restrict__ probs,
            const KIO *__restrict__ io, const T *__restrict__ tables, int it,
            const int *__restrict__ stop, int *__restrict__ status) {
  using S = Shape<P, NQ>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  if (*stop) return;
  const int2 tk = tasks[blockIdx.x];
  const int prob = tk.x, d = tk.y;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int g = pb.dir_group[d];
  const int nl = pb.n_levels_g[g];
  const int slots = (blockDim.x >> 6) * S::SPW;
  int *lo = reinterpret_cast<int *>(lds + S::TAB + (size_t)slots * S::SLOT_AREA);
  stage_tables<P, NQ, T>(tables, lds);
  const int32_t *lo_g = pb.level_off + (size_t)g * (pb.n_levels + 1);
  for (int i = threadIdx.x; i <= nl; i += blockDim.x) lo[i] = lo_g[i];
  __syncthreads();
  const int2 *dsc = pb.desc_ef + (size_t)g * pb.ne;
  const int4 *dnb = pb.desc_nb + (size_t)g * pb.ne;
  const int lane = threadIdx.x & 63;
  const int r = lane & (S::SLOT - 1);
  const int slot = (threadIdx.x >> 6) * S::SPW + lane / S::SLOT;

  // position of this slot's next solve: level L, index t
  auto fetch = [&](SolveIn<P, NQ, T> &in, int L, int t) {
    in.valid = L < nl && t < lo[L + 1];
    in.e = 0;
    in.flags = 0;
    in.nb[0] = in.nb[1] = in.nb[2] = in.nb[3] = -1;
    if (in.valid) {
      const int2 ef = dsc[t];
      const int4 nb = dnb[t];
      in.e = ef.x;
      in.flags = ef.y;
      in.nb[0] = nb.x;
      in.nb[1] = nb.y;
      in.nb[2] = nb.z;
      in.nb[3] = nb.w;
    }
    load_inputs<P, NQ, T>(in, d, pb, pio, it, r);
  };

  SolveIn<P, NQ, T> cur, nxt;
  int L = 0, base = 0;
  fetch(cur, 0, slot);
  while (L < nl) {
    // the round after (L, base)
    int L2 = L, base2 = base + slots;
    if (base2 >= lo[L + 1]) {
      L2 = L + 1;
      base2 = L2 < nl ? lo[L2] : 0;
    }
    fetch(nxt, L2, base2 + slot);
    solve_from<P, NQ, T, PIVOT>(cur, d, pb, pio, lds, r, slot, status);
    if (L2 != L) __syncthreads();  // the level's fluxes are upwind values of the next
    cur = nxt;
    L = L2;
    base = base2;
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

// Largest multiple of 64 threads <= want whose LDS fits in lds_max bytes.
template <int P, int NQ>
int fit_block(bool fp32, int want, size_t lds_max, int extra_ints, size_t *bytes) {
  using S = Shape<P, NQ>;
  for (int block = want; block >= 64; block -= 64) {
    const int slots = (block / 64) * S::SPW;
    const size_t b = fp32 ? lds_bytes<float>(S::TAB, S::SLOT_AREA, slots, extra_ints)
                          : lds_bytes<double>(S::TAB, S::SLOT_AREA, slots, extra_ints);
    if (b <= lds_max) {
      *bytes = b;
      return block;
    }
  }
  return 0;
}

template <int P, int NQ, typename T, bool PIVOT>
hipError_t launch_level_t(const SweepLaunch &L) {
  size_t bytes = 0;
  const int block = fit_block<P, NQ>(L.fp32, L.block > 256 ? 256 : L.block, L.lds_max, 0, &bytes);
  if (block == 0) return hipErrorInvalidValue;
  const int per_block = (block / 64) * Shape<P, NQ>::SPW;
  const int grid = (L.count + per_block - 1) / per_block;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_sweep_level<P, NQ, T, PIVOT>), dim3(grid), dim3(block), bytes, L.stream, L.list,
                     L.count, L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
  return hipGetLastError();
}

template <int P, int NQ, typename T, bool PIVOT>
hipError_t launch_dir_t(const SweepLaunch &L) {
  if (L.count == 0) return hipSuccess;
  constexpr int SLOT = Shape<P, NQ>::SLOT;
  const int maxb = dir_block_max<P, NQ, T>();
  int block = ((L.width * SLOT + 63) / 64) * 64;
  block = block < 64 ? 64 : (block > maxb ? maxb : block);
  size_t bytes = 0;
  block = fit_block<P, NQ>(L.fp32, block, L.lds_max, L.max_levels + 1, &bytes);
  if (block == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_dir<P, NQ, T, PIVOT>), dim3(L.count), dim3(block), bytes, L.stream, L.list,
                     L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
  return hipGetLastError();
}

template <int P, int NQ, bool DIR>
hipError_t launch_pq(const SweepLaunch &L) {
  if (DIR) {
    if (L.fp32) return L.pivot ? launch_dir_t<P, NQ, float, true>(L) : launch_dir_t<P, NQ, float, false>(L);
    return L.pivot ? launch_dir_t<P, NQ, double, true>(L) : launch_dir_t<P, NQ, double, false>(L);
  }
  if (L.fp32) return L.pivot ? launch_level_t<P, NQ, float, true>(L) : launch_level_t<P, NQ, float, false>(L);
  return L.pivot ? launch_level_t<P, NQ, double, true>(L) : launch_level_t<P, NQ, double, false>(L);
}

template <int P, bool DIR>
hipError_t launch_p(const SweepLaunch &L) {
  switch (L.nq - P) {
    case 1: return launch_pq<P, P + 1, DIR>(L);
    case 2: return launch_pq<P, P + 2, DIR>(L);
    case 3: return launch_pq<P, P + 3, DIR>(L);
    default: return hipErrorInvalidValue;
  }
}

template <bool DIR>
hipError_t launch_sweep(const SweepLaunch &L) {
  switch (L.p) {
    case 1: return launch_p<1, DIR>(L);
    case 2: return launch_p<2, DIR>(L);
    case 3: return launch_p<3, DIR>(L);
    case 4: return launch_p<4, DIR>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_sweep_level(const SweepLaunch &L) { return launch_sweep<false>(L); }
hipError_t launch_sweep_dir(const SweepLaunch &L) { return launch_sweep<true>(L); }

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

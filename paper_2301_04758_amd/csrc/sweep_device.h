// Device code of the DG S_N sweep kernels (templates shared by the per-degree
// translation units).
//
// Work mapping: a "slot" of SLOT lanes (the power of two >= n = (p+1)^2,
// aligned inside one 64-wide wavefront) owns one element-direction solve;
// lane r owns row r (test function r) of the local system.  One solve:
//   1. inputs: the lanes of the slot load the element's data, a few values
//      per lane, all loads independent (the direction-resident schedule
//      issues them one solve ahead);
//   2. staging: those values go to the slot's private LDS area (wave-local,
//      no work-group barrier);
//   3. assembly of row r, by one of two exact evaluations of the same
//      quadrature:
//      - general elements: the sum over volume points of the geometry
//        factors (w J and w adj(F)) times the basis tables, and over face
//        points of w n ds;
//      - affine elements (constant J and adj(F), straight faces): J and
//        adj(F) leave the quadrature, so the row is sigma_t J Mhat -
//        (adj(F) Omega)_xi Ghat_xi - (adj(F) Omega)_eta Ghat_eta with
//        reference matrices shared by all elements, and each face term is
//        (Omega . N_F) times the 1D face mass matrix;
//      inflow traces come from the upwind element's face nodes
//      (Gauss-Lobatto nodes include the element boundary, so a face trace is
//      the p+1 face-node values, read in reversed order because the two
//      sides run the shared face in opposite senses);
//   4. solve: Gauss-Jordan elimination with normalised pivot rows across the
//      slot's lanes, so that each lane ends with one unknown.  With partial
//      pivoting the pivot lane is one unsigned max of packed (magnitude,
//      lane) keys by DPP lane moves and the pivot row goes through the slot's
//      LDS area; without pivoting (used only when every face of the mesh is
//      straight and sigma_t > 0, so that the local matrix has a positive
//      definite symmetric part) lane k broadcasts row k by a DPP row
//      broadcast or an LDS swizzle, with no LDS round trip.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <type_traits>

#include "kernels.h"

namespace vefk {

namespace {

constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)

// Assembly/solve modes of a kernel variant.
enum : int {
  MODE_GENERAL_PIVOT = 0,
  MODE_GENERAL_NOPIVOT = 1,
  MODE_AFFINE_NOPIVOT = 2,
  MODE_AFFINE_PIPELINE = 3,  // direction-resident schedule only, p <= 2
  MODE_GENERAL_PIPELINE = 4, // the same for straight-sided bilinear elements (m = 1)
  MODE_AFFINE_LU = 5,        // affine, pivot-free, p >= 3: row-set LU with fused broadcasts
  MODE_GENERAL_MAT = 6,      // general elements, p = 3: precomputed element matrices, per-solve pivoting choice
  MODE_KIND = 7,             // mask of the kernel kind above
  MODE_FIX = 8               // flag: negative-flux fixup after each local solve
};

template <int P, int NQ>
struct Shape {
  static constexpr int P1 = P + 1;
  static constexpr int N = P1 * P1;
  static constexpr int Q = NQ * NQ;
  static constexpr int SLOT = N <= 4 ? 4 : (N <= 8 ? 8 : (N <= 16 ? 16 : 32));
  static constexpr int SPW = 64 / SLOT;
  // general path: per-lane shares of the element inputs
  static constexpr int GV = (5 * Q + SLOT - 1) / SLOT;
  static constexpr int GF = (8 * NQ + SLOT - 1) / SLOT;
  static constexpr int QD = (Q + SLOT - 1) / SLOT;
  // general path LDS: tables V, Dx, Dy [Q][n] and F [nq][p+1], then one area per slot
  static constexpr int TAB = 3 * Q * N + NQ * P1;
  static constexpr int OFF_GEO = 0;                 // [Q][5]
  static constexpr int OFF_GF = OFF_GEO + 5 * Q;    // [4][NQ][2]
  static constexpr int OFF_SRC = OFF_GF + 8 * NQ;   // [Q] source at volume points
  static constexpr int OFF_S = OFF_SRC + Q;         // [N] nodal source coefficients
  static constexpr int OFF_PIV = ((OFF_S + N + 1) / 2) * 2;  // [N + 1] pivot row + rhs
  static constexpr int SLOT_AREA = ((OFF_PIV + N + 1 + 1) / 2) * 2;
  // element-matrix path: face matrices [4][2][P1][P1], traces [4][P1], nodal
  // source [N], pivot row [N + 1]
  static constexpr int OFF_S_M = 8 * P1 * P1 + 4 * P1;
  static constexpr int OFF_PIV_M = ((OFF_S_M + N + 1) / 2) * 2;
  static constexpr int SLOT_AREA_M = ((OFF_PIV_M + N + 1 + 1) / 2) * 2;
  static constexpr int QU = P <= 2 ? Q : 1;  // volume loop fully unrolled for small elements
  // affine path: 16 values per element (J, adj(F), four face chords)
  static constexpr int GA = (16 + SLOT - 1) / SLOT;
  // tables Mhat^T, Ghat_xi^T, Ghat_eta^T [n][n], face mass [p+1][p+1],
  // w V [Q][n] (direction-dependent source), w L [nq][p+1] (boundary data)
  static constexpr int A_MT = 0, A_GX = N * N, A_GY = 2 * N * N, A_M1 = 3 * N * N;
  static constexpr int A_WV = A_M1 + P1 * P1, A_WL = A_WV + Q * N, A_GD1 = A_WL + NQ * P1;
  static constexpr int TAB_A = A_GD1 + P1 * P1;
  static constexpr int AOFF_G = 0, AOFF_S = 16, AOFF_QD = 16 + N;
  static constexpr int AOFF_PIV = ((AOFF_QD + Q + 1) / 2) * 2;
  static constexpr int SLOT_AREA_A = ((AOFF_PIV + N + 1 + 1) / 2) * 2;
};

template <int P, int NQ, int MODE>
struct Lds {
  using S = Shape<P, NQ>;
  static constexpr int TAB = (MODE & MODE_KIND) == MODE_AFFINE_NOPIVOT ? S::TAB_A : S::TAB;
  static constexpr int AREA = (MODE & MODE_KIND) == MODE_AFFINE_NOPIVOT ? S::SLOT_AREA_A
                             : (MODE & MODE_KIND) == MODE_GENERAL_MAT  ? S::SLOT_AREA_M
                                                                       : S::SLOT_AREA;
};

template <typename T>
__host__ __device__ constexpr size_t lds_bytes(int tab, int slot_area, int slots, int extra_ints) {
  return sizeof(T) * ((size_t)tab + (size_t)slot_area * slots) + sizeof(int) * (size_t)extra_ints;
}

// node index of position c (counter-clockwise) along face f
// Global-memory view of a generic pointer.  Accesses through it compile to
// global_* instructions, which count only on vmcnt; flat accesses also count
// on lgkmcnt, so every wait for LDS results would wait for them too.
#define VEF_GLOBAL __attribute__((address_space(1)))
// Constant-memory view (uniform reads compile to scalar loads).
#define VEF_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ VEF_GLOBAL T *gmem(T *p) {
  return (VEF_GLOBAL T *)p;
}

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

// XCD-aware block order.  Work-groups are dealt to the 8 XCDs round-robin
// by index, and each XCD has its own L2; the level lists hold the solves of
// one element (its directions) next to each other, so giving each XCD a
// contiguous range of blocks keeps an element's data in one L2.  Block b
// runs on XCD b % 8 as its (b / 8)-th block there; the result is a bijection
// of [0, grid).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int grid) {
  const int x = b % kXcds, j = b / kXcds, q = grid / kXcds, r = grid % kXcds;
  return x * q + (x < r ? x : r) + j;
}

// face_node without branches (selects), for a runtime face
template <int P>
__device__ __forceinline__ int face_node_sel(int f, int c) {
  constexpr int P1 = P + 1;
  const int base = f == 0 ? 0 : f == 1 ? P : f == 2 ? P + P1 * P : P1 * P;
  const int step = f == 0 ? 1 : f == 1 ? P1 : f == 2 ? -1 : -P1;
  return base + step * c;
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

// Angular-flux accesses that other work-groups of the same launch may read
// (COH: the persistent schedule) are agent-scope atomic loads and stores:
// each goes to the device's coherence point by itself, so no cache-wide
// fence is needed around them.
// Loads and stores through global-address-space pointers.  A pointer taken
// from a descriptor in memory is generic, and a generic (flat) access counts
// against the LDS counter as well, so a wait for an LDS read would also wait
// for it; the streaming kernels keep loads in flight across LDS work.
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
  return *gmem(p);
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, T v) {
  *gmem(p) = v;
}

template <bool COH, typename T>
__device__ __forceinline__ T ld_psi(const T *p) {
  if constexpr (COH)
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return gload(p);
}
template <bool COH, typename T>
__device__ __forceinline__ void st_psi(T *p, T v) {
  if constexpr (COH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    gstore(p, v);
}

template <int B, int E, int S = 1, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr ((S > 0 && B < E) || (S < 0 && B > E)) {
    f(std::integral_constant<int, B>{});
    static_for<B + S, E, S>(f);
  }
}

// acc -= src[lane K of the 16-lane row] * mul, the broadcast fused into the
// multiply-add.  The s_nop provides the two wait states a DPP read needs after
// a VALU write of its source (the compiler does not insert them for asm).
template <int K>
__device__ __forceinline__ void fnma_bcast(double &acc, double src, double mul) {
  asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(src), "v"(mul), "i"(K));
}
template <int K>
__device__ __forceinline__ void fnma_bcast(float &acc, float src, float mul) {
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, -%2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(src), "v"(mul), "i"(K));
}

// Blocks of the same update over several columns J in one asm statement:
// within a block no instruction reads a register written by the one before
// it (each column's updates write different registers from those the next
// column's read), so a single s_nop at the start covers the whole block.
// fnma_bcast_2x4: columns j = 0..3, hi[j] -= bcast(lo[j]) * lh, then
// lo[j] -= bcast(lo[j]) * ll (the pivot set's rows last).
#define VEF_FMAC_DPP(OP, ACC, SRC, MUL) \
  OP " " ACC ", " SRC ", -" MUL " row_newbcast:%[k] row_mask:0xf bank_mask:0xf\n\t"
#define VEF_BCAST_2X4(OP)                                                                                    \
  "s_nop 1\n\t" VEF_FMAC_DPP(OP, "%[h0]", "%[o0]", "%[lh]") VEF_FMAC_DPP(OP, "%[o0]", "%[o0]", "%[ll]")  \
      VEF_FMAC_DPP(OP, "%[h1]", "%[o1]", "%[lh]") VEF_FMAC_DPP(OP, "%[o1]", "%[o1]", "%[ll]")              \
          VEF_FMAC_DPP(OP, "%[h2]", "%[o2]", "%[lh]") VEF_FMAC_DPP(OP, "%[o2]", "%[o2]", "%[ll]")          \
              VEF_FMAC_DPP(OP, "%[h3]", "%[o3]", "%[lh]") VEF_FMAC_DPP(OP, "%[o3]", "%[o3]", "%[ll]")
#define VEF_BCAST_1X8(OP)                                                                                    \
  "s_nop 1\n\t" VEF_FMAC_DPP(OP, "%[o0]", "%[o0]", "%[ll]") VEF_FMAC_DPP(OP, "%[o1]", "%[o1]", "%[ll]")  \
      VEF_FMAC_DPP(OP, "%[o2]", "%[o2]", "%[ll]") VEF_FMAC_DPP(OP, "%[o3]", "%[o3]", "%[ll]")              \
          VEF_FMAC_DPP(OP, "%[o4]", "%[o4]", "%[ll]") VEF_FMAC_DPP(OP, "%[o5]", "%[o5]", "%[ll]")          \
              VEF_FMAC_DPP(OP, "%[o6]", "%[o6]", "%[ll]") VEF_FMAC_DPP(OP, "%[o7]", "%[o7]", "%[ll]")

template <int K, typename T>
__device__ __forceinline__ void fnma_bcast_2x4(T &o0, T &o1, T &o2, T &o3, T &h0, T &h1, T &h2, T &h3, T ll, T lh) {
  if constexpr (sizeof(T) == 8)
    asm(VEF_BCAST_2X4("v_fmac_f64_dpp")
        : [o0] "+v"(o0), [o1] "+v"(o1), [o2] "+v"(o2), [o3] "+v"(o3), [h0] "+v"(h0), [h1] "+v"(h1), [h2] "+v"(h2),
          [h3] "+v"(h3)
        : [ll] "v"(ll), [lh] "v"(lh), [k] "i"(K));
  else
    asm(VEF_BCAST_2X4("v_fmac_f32_dpp")
        : [o0] "+v"(o0), [o1] "+v"(o1), [o2] "+v"(o2), [o3] "+v"(o3), [h0] "+v"(h0), [h1] "+v"(h1), [h2] "+v"(h2),
          [h3] "+v"(h3)
        : [ll] "v"(ll), [lh] "v"(lh), [k] "i"(K));
}
template <int K, typename T>
__device__ __forceinline__ void fnma_bcast_1x8(T &o0, T &o1, T &o2, T &o3, T &o4, T &o5, T &o6, T &o7, T ll) {
  if constexpr (sizeof(T) == 8)
    asm(VEF_BCAST_1X8("v_fmac_f64_dpp")
        : [o0] "+v"(o0), [o1] "+v"(o1), [o2] "+v"(o2), [o3] "+v"(o3), [o4] "+v"(o4), [o5] "+v"(o5), [o6] "+v"(o6),
          [o7] "+v"(o7)
        : [ll] "v"(ll), [k] "i"(K));
  else
    asm(VEF_BCAST_1X8("v_fmac_f32_dpp")
        : [o0] "+v"(o0), [o1] "+v"(o1), [o2] "+v"(o2), [o3] "+v"(o3), [o4] "+v"(o4), [o5] "+v"(o5), [o6] "+v"(o6),
          [o7] "+v"(o7)
        : [ll] "v"(ll), [k] "i"(K));
}

// Natural-order LU of the augmented rows [A | b] of one solve held RS rows
// per lane of a 16-lane slot (row l + s H of set s in lane l), then the back
// substitution: on return A[s][N] holds U x (the unknown times its pivot) and
// idg[s] the reciprocal pivot of row l + s H, so x = A[s][N] * idg[s].  Step
// K broadcasts pivot row K from its lane with row_newbcast fused into each
// update; the multipliers of the mixed set (the set holding row K) are zero
// for the rows at or above it, and its pivot and multipliers are cleared as
// they are used, so the back substitution needs no masks.
template <int N, int RS, int H, typename T>
__device__ __forceinline__ void lu_rows(T (&A)[RS][N + 1], T (&idg)[RS], int r) {
  // LU of [A | b] in natural order
#pragma unroll
  for (int s = 0; s < RS; ++s) idg[s] = T(0);
  static_for<0, N>([&](auto kk) {
    constexpr int K = decltype(kk)::value;
    constexpr int SA = K / H, LK = K % H;
    const T inv = slot_bcast<16, LK>(recip(A[SA][K]));
    if (r == LK) idg[SA] = inv;
    T l[RS];
#pragma unroll
    for (int s = SA; s < RS; ++s) l[s] = A[s][K] * inv;
    l[SA] = r > LK ? l[SA] : T(0);
    A[SA][K] = r >= LK ? T(0) : A[SA][K];
    // the trailing columns K + 1 .. N: blocks of columns, then one at a time
    constexpr int NB = RS - SA == 2 ? 4 : RS - SA == 1 ? 8 : 1;  // columns per block
    constexpr int JB = NB > 1 ? K + 1 + ((N - K) / NB) * NB : K + 1;  // first column after the blocks
    if constexpr (NB == 4) {
      static_for<K + 1, JB, 4>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        fnma_bcast_2x4<LK>(A[SA][J], A[SA][J + 1], A[SA][J + 2], A[SA][J + 3], A[SA + 1][J], A[SA + 1][J + 1],
                           A[SA + 1][J + 2], A[SA + 1][J + 3], l[SA], l[SA + 1]);
      });
    } else if constexpr (NB == 8) {
      static_for<K + 1, JB, 8>([&](auto jj) {
        constexpr int J = decltype(jj)::value;
        fnma_bcast_1x8<LK>(A[SA][J], A[SA][J + 1], A[SA][J + 2], A[SA][J + 3], A[SA][J + 4], A[SA][J + 5],
                           A[SA][J + 6], A[SA][J + 7], l[SA]);
      });
    }
    static_for<JB, N + 1>([&](auto jj) {
      constexpr int J = decltype(jj)::value;
      static_for<SA + 1, RS>([&](auto ss) { fnma_bcast<LK>(A[decltype(ss)::value][J], A[SA][J], l[decltype(ss)::value]); });
      fnma_bcast<LK>(A[SA][J], A[SA][J], l[SA]);
    });
  });
  // back substitution U x = y on the right-hand side column
  static_for<N - 1, -1, -1>([&](auto ii) {
    constexpr int I = decltype(ii)::value;
    constexpr int SA = I / H, LI = I % H;
    const T t = A[SA][N] * idg[SA];
    static_for<0, SA + 1>([&](auto ss) { fnma_bcast<LI>(A[decltype(ss)::value][N], t, A[decltype(ss)::value][I]); });
  });
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

// Negative-flux fixup of one solve held one unknown per lane (x, with its
// balance weight c): when some unknown of the slot is negative, negatives
// become zero and the rest is scaled by (c . x) / (c . x+), which keeps the
// element's particle balance c . x; a slot without negative unknowns is left
// alone.  c_j = sigma_t int phi_j + outflow int (Omega . n) phi_j, the column
// sums of the local matrix (the streaming columns sum to zero).  Wave-uniform
// early exit: the reductions run only when some lane has a negative value.
template <int SLOT, typename T>
__device__ __forceinline__ void zero_and_scale_slot(T &x, T c, bool row_ok) {
  const bool neg = row_ok && x < T(0);
  if (__builtin_amdgcn_ballot_w64(neg) == 0) return;
  T cx = row_ok ? c * x : T(0);
  T cp = (row_ok && x > T(0)) ? c * x : T(0);
  int nneg = neg ? 1 : 0;
#pragma unroll
  for (int m = 1; m < SLOT; m <<= 1) {
    cx += __shfl_xor(cx, m);
    cp += __shfl_xor(cp, m);
    nneg += __shfl_xor(nneg, m);
  }
  if (nneg > 0 && row_ok) {
    const T alpha = (cx > T(0) && cp > T(0)) ? cx / cp : T(0);
    x = x > T(0) ? alpha * x : T(0);
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
__device__ __forceinline__ void load_one(SolveIn<P, NQ, T> &in, int d, const KProb &pb,
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
template <int P, int NQ, typename T, bool PIVOT, bool FIX, bool COH = false>
__device__ __forceinline__ void solve_one(const SolveIn<P, NQ, T> &in, int d, const KProb &pb,
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
      for (int c = 0; c < P1; ++c) tr[f][c] = ld_psi<COH>(up + face_node<P>(f2, P - c));
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
  // A[(c,d)] = sum_q coef_q V_(c,d)(q) with the tensor basis V_(c,d)(qx,qy) =
  // v1[qx][c] v1[qy][d] (v1 = the face table sF), summed by factors:
  // first over qx for each qy (P1 values), then over qy.
#pragma unroll S::QU
  for (int qy = 0; qy < NQ; ++qy) {
    T coef[NQ];
#pragma unroll
    for (int qx = 0; qx < NQ; ++qx) {
      const int q = qx + NQ * qy;
      const T wJ = g5[5 * q], a00 = g5[5 * q + 1], a01 = g5[5 * q + 2], a10 = g5[5 * q + 3], a11 = g5[5 * q + 4];
      const T gx = a00 * ox + a01 * oy;
      const T gy = a10 * ox + a11 * oy;
      const T li = sV[q * N + rr];
      coef[qx] = st * wJ * li - (gx * sDx[q * N + rr] + gy * sDy[q * N + rr]);
      rhs += wJ * li * srcq[q];
    }
    T trow[P1];
#pragma unroll
    for (int c = 0; c < P1; ++c) {
      T acc = T(0);
#pragma unroll
      for (int qx = 0; qx < NQ; ++qx) acc += coef[qx] * sF[qx * P1 + c];
      trow[c] = acc;
    }
#pragma unroll
    for (int dd = 0; dd < P1; ++dd) {
      const T vd = sF[qy * P1 + dd];
#pragma unroll
      for (int c = 0; c < P1; ++c) A[c + P1 * dd] += vd * trow[c];
    }
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
    } else if (pb.pointwise) {
      // an inflow face with pointwise upwinding: each point takes the
      // upwind value where Omega . n < 0 and the element's own trace (a
      // matrix term) elsewhere
      const double *bc = (in.nb[f] < 0 && pio.psi_bc) ? pio.psi_bc + ((size_t)d * pb.nbf + (-in.nb[f] - 1)) * NQ
                                                      : nullptr;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T on = ox * gf[2 * q] + oy * gf[2 * q + 1];
        const T t = on * sF[q * P1 + pos];
        if (!(on < T(0))) {
#pragma unroll
          for (int c = 0; c < P1; ++c) A[face_node<P>(f, c)] += t * sF[q * P1 + c];
        } else if (in.nb[f] >= 0) {
          T ph = T(0);
#pragma unroll
          for (int c = 0; c < P1; ++c) ph += tr[f][c] * sF[q * P1 + c];
          rhs -= t * ph;
        } else if (bc) {
          rhs -= t * static_cast<T>(bc[q]);
        }
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

  // elimination; lane r ends with unknown my_k in rhs
  int my_k = r;
  if constexpr (PIVOT && SLOT == 16 && N == 16) {
    // a solve certified for elimination in natural order (flags bit 12
    // clear: see the plan) takes the LU with fused broadcasts, the others
    // Gauss-Jordan with partial pivoting; the choice is per slot, and both
    // stay inside the slot's DPP row and LDS area
    if (!((in.flags >> 12) & 1)) {
      T A1[1][N + 1], idg[1];
#pragma unroll
      for (int j = 0; j < N; ++j) A1[0][j] = A[j];
      A1[0][N] = rhs;
      lu_rows<N, 1, 16, T>(A1, idg, r);
      rhs = A1[0][N] * idg[0];
    } else {
      bool active = row_ok;
      gj_pivot<SLOT, N, 0, T>(A, rhs, r, active, my_k, area + S::OFF_PIV);
    }
  } else if constexpr (PIVOT) {
    bool active = row_ok;
    gj_pivot<SLOT, N, 0, T>(A, rhs, r, active, my_k, area + S::OFF_PIV);
  } else {
    gj_nopivot<SLOT, N, 0, T>(A, rhs, r);
  }
  if constexpr (FIX) {
    // balance weight of unknown rr, recomputed here (rare path) from the
    // geometry still in LDS: sigma_t int phi_rr + outflow int (Omega.n) phi_rr
    T cr = T(0);
    if (row_ok) {
      T cv = T(0);
      for (int q = 0; q < Q; ++q) cv += g5[5 * q] * sV[q * N + rr];
      cr = static_cast<T>(pb.sig[2 * e]) * cv;
      for (int f = 0; f < 4; ++f) {
        const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
        const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
        if (!on_face || ((mask >> f) & 1u)) continue;
        const T *gf = area + S::OFF_GF + f * NQ * 2;
        for (int q = 0; q < NQ; ++q) cr += (ox * gf[2 * q] + oy * gf[2 * q + 1]) * sF[q * P1 + pos];
      }
    }
    if constexpr (PIVOT) {  // lane r holds unknown my_k: fetch its weight
      T *cw = area + S::OFF_PIV;
      if (row_ok) cw[r] = cr;
      wave_sync_lds();
      cr = cw[my_k];
      __builtin_amdgcn_wave_barrier();
    }
    zero_and_scale_slot<SLOT, T>(rhs, cr, row_ok);
  }
  if (row_ok) {
    T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
    st_psi<COH>(out + my_k, rhs);
    if (!__builtin_isfinite(rhs)) atomicOr(status, 1);  // non-finite unknown
  }
}

// ---------------------------------------------------------------------------
// General elements with precomputed element matrices (degree 3).  The
// direction-independent parts of the local system are formed once per
// element (k_elem_mat, matrix cores): the mass matrix M_ij = int phi_i phi_j,
// the streaming matrices G^x_ij, G^y_ij = int (dphi_i / dx or dy) phi_j
// (adj(F)^T grad^ phi_i at the volume points), and per face f the face mass
// weighted by each normal component, F^x_f, F^y_f [p+1][p+1] (w_s n ds at
// the face points).  A solve then assembles
//   A = sigma_t M - Omega_x G^x - Omega_y G^y + sum over outflow faces of
//       (Omega_x F^x_f + Omega_y F^y_f) on the face nodes,
//   b = M s - sum over inflow faces of (Omega_x F^x_f + Omega_y F^y_f) times
//       the upwind trace (boundary data by face quadrature),
// three multiply-adds per entry in place of the quadrature sums.  Layout per
// element: M, G^x, G^y [n][n] row major, then [4][2][p+1][p+1].
// ---------------------------------------------------------------------------
template <int P>
struct EMat {
  static constexpr int P1 = P + 1, N = P1 * P1;
  static constexpr int OFF_GX = N * N, OFF_GY = 2 * N * N, OFF_F = 3 * N * N;
  static constexpr int SIZE = 3 * N * N + 8 * P1 * P1;  // values per element
};

// ORD: a solve not certified for elimination in natural order assembles its
// rows in the partial-pivoting order formed for it before the sweep (row
// piv_perm[16 pix + r] on lane r) and eliminates in natural order; without
// ORD such a solve runs Gauss-Jordan with partial pivoting.
template <int P, int NQ, typename T, bool ORD = false>
struct SolveInM {
  int e, flags;  // flags as SolveIn
  int nb[4];
  bool valid;
  int pix;  // ORD: the solve's entry of piv_perm
  int rr;   // the row of the local matrix this lane assembles
  T s;      // nodal source at node r
};

template <int P, int NQ, typename T, bool ORD>
__device__ __forceinline__ void load_one(SolveInM<P, NQ, T, ORD> &in, int d, const KProb &pb, const KIO &pio,
                                         int it, int r) {
  constexpr int N = (P + 1) * (P + 1);
  (void)d;
  in.rr = r;
  if (!in.valid) return;
  if constexpr (ORD) {
    if ((in.flags >> 12) & 1) in.rr = gload(pb.piv_perm + (size_t)in.pix * 16 + r) & 15;
  }
  const int e = in.e;
  const double *phi = it == 0 ? pio.phi_in : pio.mom;
  T sv = T(0);
  if (r < N) {
    if (phi) sv = static_cast<T>(gload(pb.sig + 2 * e + 1) * kInv4Pi) * static_cast<T>(gload(phi + (size_t)e * N + r));
    if (pio.q_iso) sv += static_cast<T>(gload(pio.q_iso + (size_t)e * N + r));
  }
  in.s = sv;
}

template <int P, int NQ, typename T, bool PIVOT, bool FIX, bool COH = false, bool ORD>
__device__ __forceinline__ void solve_one(const SolveInM<P, NQ, T, ORD> &in, int d, const KProb &pb,
                                          const KIO &pio, T *lds, int r, int slot, int *status) {
  using S = Shape<P, NQ>;
  using EM = EMat<P>;
  constexpr int P1 = S::P1, N = S::N, Q = S::Q, SLOT = S::SLOT;
  static_assert(N == 16 && SLOT == 16, "element matrices: degree 3");
  // the face table F [nq][P1], read from the double tables (boundary data
  // only), so that the level kernel stages no tables
  const double *sF = pb.tab_d + 3 * Q * N;
  T *area = lds + S::TAB + (size_t)slot * S::SLOT_AREA_M;
  const int ne = pb.ne;
  const int e = in.e;
  const bool valid = in.valid;
  const bool row_ok = valid && r < N;
  const int rr = in.rr;  // r, or the pivot order's row (N == SLOT)
  const int a = rr % P1, b = rr / P1;
  const unsigned mask = valid ? (unsigned)in.flags & 15u : 0u;

  // the lane's rows of M, G^x, G^y (entry (i, j) at ((j / W) 16 + i) W + j %
  // W: the slot's 16 lanes read 16 W consecutive values per 16-byte load)
  const T *em = static_cast<const T *>(pb.emat) + (size_t)(valid ? e : 0) * EM::SIZE;
  T mr[N], gx[N], gy[N];
  {
    constexpr int W = 16 / sizeof(T);
    typedef T VW __attribute__((ext_vector_type(W)));
#pragma unroll
    for (int jj = 0; jj < N / W; ++jj) {
      const int at = (jj * 16 + rr) * W;
      const VW vm = gload(reinterpret_cast<const VW *>(em + at));
      const VW vx = gload(reinterpret_cast<const VW *>(em + EM::OFF_GX + at));
      const VW vy = gload(reinterpret_cast<const VW *>(em + EM::OFF_GY + at));
#pragma unroll
      for (int w = 0; w < W; ++w) {
        mr[W * jj + w] = vm[w];
        gx[W * jj + w] = vx[w];
        gy[W * jj + w] = vy[w];
      }
    }
  }
  // the face matrices [4][2][P1][P1] and the upwind traces [4][P1] go
  // through the slot's LDS area, each lane loading a share, so that they hold
  // no registers across the assembly
  constexpr int FM = 8 * P1 * P1, A_FM = 0, A_TR = FM;
  static_assert(A_TR + 4 * P1 <= S::OFF_S_M && P1 * 4 == 16, "element-matrix staging layout");
  T fm[FM / 16];
#pragma unroll
  for (int k = 0; k < FM / 16; ++k) fm[k] = gload(em + EM::OFF_F + r + 16 * k);
  T trv = T(0);
  {
    // trace entry r: face r / P1, face node r % P1 (P1 = 4: one per lane)
    const int f = r / P1, c = r % P1;
    const int n0 = in.nb[0], n1 = in.nb[1], n2 = in.nb[2], n3 = in.nb[3];  // values, not addresses, selected
    const int u = f == 0 ? n0 : f == 1 ? n1 : f == 2 ? n2 : n3;
    if (valid && ((mask >> f) & 1u) && u >= 0) {
      const int f2 = (in.flags >> (4 + 2 * f)) & 3;
      trv = ld_psi<COH>(static_cast<const T *>(pio.psi) + ((size_t)d * ne + u) * N + face_node_sel<P>(f2, P - c));
    }
  }
#pragma unroll
  for (int k = 0; k < FM / 16; ++k) area[A_FM + r + 16 * k] = fm[k];
  area[A_TR + r] = trv;
  if (r < N) area[S::OFF_S_M + r] = in.s;
  wave_sync_lds();

  const T ox = static_cast<T>(gload(pb.omega + 2 * d));
  const T oy = static_cast<T>(gload(pb.omega + 2 * d + 1));
  const T st = static_cast<T>(gload(pb.sig + 2 * (valid ? e : 0)));
  T A[N];
  T rhs = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    A[j] = st * mr[j] - (ox * gx[j] + oy * gy[j]);
    rhs += mr[j] * area[S::OFF_S_M + j];
  }
  if (pio.q_dir && row_ok) {
    // direction-dependent source at the volume points: int phi_r q_dir (V
    // from the double tables: only the face table is staged)
    const T *g5 = static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5;
    const double *qd = pio.q_dir + ((size_t)d * ne + e) * Q;
    T acc = T(0);
    for (int q = 0; q < Q; ++q)
      acc += gload(g5 + 5 * q) * static_cast<T>(gload(pb.tab_d + q * N + rr)) * static_cast<T>(gload(qd + q));
    rhs += acc;
  }
  T cw = T(0);  // outflow part of the balance weight (fixup)
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
    const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
    if (!(row_ok && on_face)) continue;
    const T *fxr = area + A_FM + (2 * f) * P1 * P1 + pos * P1;
    const T *fyr = fxr + P1 * P1;
    if (!((mask >> f) & 1u)) {
#pragma unroll
      for (int c = 0; c < P1; ++c) {
        const T t = ox * fxr[c] + oy * fyr[c];
        A[face_node<P>(f, c)] += t;
        if constexpr (FIX) cw += t;
      }
    } else if (in.nb[f] >= 0) {
#pragma unroll
      for (int c = 0; c < P1; ++c) rhs -= (ox * fxr[c] + oy * fyr[c]) * area[A_TR + f * P1 + c];
    } else if (pio.psi_bc) {
      const T *gf = static_cast<const T *>(pb.geo_f) + (size_t)e * 8 * NQ + f * NQ * 2;
      const double *bc = pio.psi_bc + ((size_t)d * pb.nbf + (-in.nb[f] - 1)) * NQ;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const T on = ox * gload(gf + 2 * q) + oy * gload(gf + 2 * q + 1);
        rhs -= on * static_cast<T>(gload(sF + q * P1 + pos)) * static_cast<T>(gload(bc + q));
      }
    }
  }

  // elimination: the LU with fused broadcasts in natural order (certified
  // solves; with ORD every solve, its rows already in pivoting order), or
  // Gauss-Jordan with partial pivoting (see the general solve); lane r ends
  // with unknown my_k
  int my_k = r;
  if (!PIVOT || ORD || !((in.flags >> 12) & 1)) {
    T A1[1][N + 1], idg[1];
#pragma unroll
    for (int j = 0; j < N; ++j) A1[0][j] = A[j];
    A1[0][N] = rhs;
    lu_rows<N, 1, 16, T>(A1, idg, r);
    rhs = A1[0][N] * idg[0];
  } else if constexpr (PIVOT && !ORD) {
    bool active = row_ok;
    gj_pivot<SLOT, N, 0, T>(A, rhs, r, active, my_k, area + S::OFF_PIV_M);
  }
  if constexpr (FIX) {
    // balance weight of unknown rr: sigma_t int phi_rr (a row sum of M, the
    // basis summing to one) plus the outflow terms
    T cr = T(0);
    if (row_ok) {
      T sm = T(0);
#pragma unroll
      for (int j = 0; j < N; ++j) sm += mr[j];
      cr = st * sm + cw;
    }
    if constexpr (PIVOT) {  // the weight of row rr, wanted for unknown my_k
      T *cwl = area + S::OFF_PIV_M;
      if (row_ok) cwl[rr] = cr;
      wave_sync_lds();
      cr = cwl[my_k];
      __builtin_amdgcn_wave_barrier();
    }
    zero_and_scale_slot<SLOT, T>(rhs, cr, row_ok);
  }
  if (row_ok) {
    T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
    st_psi<COH>(out + my_k, rhs);
    if (!__builtin_isfinite(rhs)) atomicOr(status, 1);  // non-finite unknown
  }
}

// Per-lane inputs of one solve on an affine element.
template <int P, int NQ, typename T>
struct SolveInA {
  using S = Shape<P, NQ>;
  int e, flags;
  int nb[4];
  bool valid;
  T g[S::GA];
  T s;
  T qd[S::QD];
};

template <int P, int NQ, typename T>
__device__ __forceinline__ void load_one(SolveInA<P, NQ, T> &in, int d, const KProb &pb, const KIO &pio,
                                         int it, int r) {
  using S = Shape<P, NQ>;
  constexpr int N = S::N, Q = S::Q, SLOT = S::SLOT;
  const int e = in.e;
  if (!in.valid) return;
  const T *ga = static_cast<const T *>(pb.geo_a) + (size_t)e * 16;
#pragma unroll
  for (int k = 0; k < S::GA; ++k) {
    const int i = r + k * SLOT;
    in.g[k] = i < 16 ? ga[i] : T(0);
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

// Solve on an affine element (see the file comment); pivot-free.
template <int P, int NQ, typename T, bool PIVOT, bool FIX, bool COH = false>
__device__ __forceinline__ void solve_one(const SolveInA<P, NQ, T> &in, int d, const KProb &pb,
                                          const KIO &pio, T *lds, int r, int slot, int *status) {
  using S = Shape<P, NQ>;
  constexpr int P1 = S::P1, N = S::N, Q = S::Q, SLOT = S::SLOT;
  static_assert(!PIVOT, "the affine path is pivot-free");
  const T *M1 = lds + S::A_M1;
  const T *WV = lds + S::A_WV;
  const T *WL = lds + S::A_WL;
  T *area = lds + S::TAB_A + (size_t)slot * S::SLOT_AREA_A;
  const int ne = pb.ne;
  const int e = in.e;
  const bool valid = in.valid;
  const bool row_ok = valid && r < N;
  const int rr = r < N ? r : N - 1;
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
      for (int c = 0; c < P1; ++c) tr[f][c] = ld_psi<COH>(up + face_node<P>(f2, P - c));
    }
  }

  // staging (wave-local)
#pragma unroll
  for (int k = 0; k < S::GA; ++k) {
    const int i = r + k * SLOT;
    if (i < 16) area[S::AOFF_G + i] = in.g[k];
  }
  if (r < N) area[S::AOFF_S + r] = in.s;
  if (pio.q_dir) {
#pragma unroll
    for (int k = 0; k < S::QD; ++k) {
      const int q = r + k * SLOT;
      if (q < Q) area[S::AOFF_QD + q] = in.qd[k];
    }
  }
  wave_sync_lds();

  // assembly of row r
  const T ox = static_cast<T>(pb.omega[2 * d]);
  const T oy = static_cast<T>(pb.omega[2 * d + 1]);
  const T st = static_cast<T>(pb.sig[2 * (valid ? e : 0)]);
  const T *g = area + S::AOFF_G;
  const T J = g[0];
  const T stJ = st * J;
  const T gx = g[1] * ox + g[2] * oy;
  const T gy = g[3] * ox + g[4] * oy;
  // Row rr = (a, b) of A = stJ M - gx Gx - gy Gy from the 1D factors:
  // M = m (x) m, Gx = gd (x) m, Gy = m (x) gd (test index first), so
  // A[(a,b)][(c,d)] = m_bd (stJ m_ac - gx gd_ac) - gd_bd (gy m_ac).
  const T *m1 = lds + S::A_M1;
  const T *gdt = lds + S::A_GD1;
  T mb[P1], gb[P1], Xa[P1], Ya[P1];
#pragma unroll
  for (int c = 0; c < P1; ++c) {
    const T mac = m1[a * P1 + c];
    Xa[c] = stJ * mac - gx * gdt[a * P1 + c];
    Ya[c] = gy * mac;
    mb[c] = m1[b * P1 + c];
    gb[c] = gdt[b * P1 + c];
  }
  T A[N];
  T rhs = T(0);
#pragma unroll
  for (int dd = 0; dd < P1; ++dd) {
    T acc = T(0);
#pragma unroll
    for (int c = 0; c < P1; ++c) {
      A[c + P1 * dd] = mb[dd] * Xa[c] - gb[dd] * Ya[c];
      acc += m1[a * P1 + c] * area[S::AOFF_S + c + P1 * dd];
    }
    rhs += mb[dd] * acc;  // (m (x) m) s, summed over (c, d)
  }
  rhs *= J;
  if (pio.q_dir) {
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) acc += WV[q * N + rr] * area[S::AOFF_QD + q];
    rhs += J * acc;
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
    const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
    if (!(row_ok && on_face)) continue;
    const T on = ox * g[5 + 2 * f] + oy * g[6 + 2 * f];
    if (!((mask >> f) & 1u)) {
#pragma unroll
      for (int c = 0; c < P1; ++c) A[face_node<P>(f, c)] += on * M1[pos * P1 + c];
    } else if (in.nb[f] >= 0) {
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < P1; ++c) acc += M1[pos * P1 + c] * tr[f][c];
      rhs -= on * acc;
    } else if (pio.psi_bc) {
      const double *bc = pio.psi_bc + ((size_t)d * pb.nbf + (-in.nb[f] - 1)) * NQ;
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc += WL[q * P1 + pos] * static_cast<T>(bc[q]);
      rhs -= on * acc;
    }
  }

  gj_nopivot<SLOT, N, 0, T>(A, rhs, r);
  if constexpr (FIX) {
    // balance weight of unknown rr (rare path): stJ (sum_c m_ac)(sum_d m_bd)
    // + outflow faces through rr: (Omega . N_f) sum_c M1[pos][c]
    T cr = T(0);
    if (row_ok) {
      T sma = T(0), smb = T(0);
      for (int c = 0; c < P1; ++c) {
        sma += m1[a * P1 + c];
        smb += m1[b * P1 + c];
      }
      cr = static_cast<T>(pb.sig[2 * e]) * area[S::AOFF_G] * sma * smb;
      for (int f = 0; f < 4; ++f) {
        const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
        const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
        if (!on_face || ((mask >> f) & 1u)) continue;
        const T on = ox * area[S::AOFF_G + 5 + 2 * f] + oy * area[S::AOFF_G + 6 + 2 * f];
        for (int c = 0; c < P1; ++c) cr += on * M1[pos * P1 + c];
      }
    }
    zero_and_scale_slot<SLOT, T>(rhs, cr, row_ok);
  }
  if (row_ok) {
    T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
    st_psi<COH>(out + r, rhs);
    if (!__builtin_isfinite(rhs)) atomicOr(status, 1);  // non-finite unknown
  }
}

template <int P, int NQ, typename T, int MODE, bool ORD = false>
using InputsOf = std::conditional_t<
    (MODE & MODE_KIND) == MODE_AFFINE_NOPIVOT, SolveInA<P, NQ, T>,
    std::conditional_t<(MODE & MODE_KIND) == MODE_GENERAL_MAT, SolveInM<P, NQ, T, ORD>, SolveIn<P, NQ, T>>>;

// Modes whose solves may pivot (per solve: see the plan's certification bit).
constexpr bool mode_pivots(int mode) {
  return (mode & MODE_KIND) == MODE_GENERAL_PIVOT || (mode & MODE_KIND) == MODE_GENERAL_MAT;
}

// Stage the tables of a variant into LDS.
template <int P, int NQ, typename T, int MODE>
__device__ __forceinline__ void stage_tables(const T *__restrict__ tables, T *lds) {
  constexpr int TAB = Lds<P, NQ, MODE>::TAB;
  // the element-matrix kernels read only the face table F (after V, Dx, Dy)
  constexpr int FIRST = (MODE & MODE_KIND) == MODE_GENERAL_MAT ? 3 * NQ * NQ * (P + 1) * (P + 1) : 0;
  for (int i = FIRST + threadIdx.x; i < TAB; i += blockDim.x) lds[i] = tables[i];
}

// Level-synchronous schedule: one launch per upwind level over the list of
// (element, direction | problem << 16) pairs of that level.
template <int P, int NQ, typename T, int MODE>
__global__ void __launch_bounds__(256)
k_sweep_level(const int4 *__restrict__ desc, int n_solves, const KProb *__restrict__ probs,
              const KIO *__restrict__ io, const T *__restrict__ tables, int it,
              const int *__restrict__ stop, int *__restrict__ status) {
  using S = Shape<P, NQ>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int r = lane & (S::SLOT - 1);
  const int slot = (threadIdx.x >> 6) * S::SPW + lane / S::SLOT;
  const int sid = xcd_block(blockIdx.x, gridDim.x) * ((blockDim.x >> 6) * S::SPW) + slot;
  InputsOf<P, NQ, T, MODE, true> in;
  in.valid = sid < n_solves;
  // the solve's descriptor, read before the stop flag so the two loads overlap
  int4 da = make_int4(0, 0, 0, 0), db = make_int4(-1, -1, -1, -1);
  if (in.valid) {
    da = desc[2 * (size_t)sid];
    db = desc[2 * (size_t)sid + 1];
  }
  if (*stop) return;
  if constexpr ((MODE & MODE_KIND) != MODE_GENERAL_MAT) {  // the element-matrix solve reads no staged table
    stage_tables<P, NQ, T, MODE>(tables, lds);
    __syncthreads();
  }
  in.valid = in.valid && da.x >= 0;  // element -1: an entry that pads a problem's solves to whole waves
  in.e = in.valid ? da.x : 0;
  // one problem per wave (the lists start each problem's solves on a whole
  // wave): its records come through the scalar cache
  const int d = da.y & 0xffff, prob = __builtin_amdgcn_readfirstlane(da.y >> 16);
  if (in.valid && (da.y >> 16) != prob) atomicOr(status, 4);  // a list that breaks that layout
  in.flags = da.z & 0xffff;  // inflow faces, neighbour faces, pivoting needed
  in.nb[0] = db.x;
  in.nb[1] = db.y;
  in.nb[2] = db.z;
  in.nb[3] = db.w;
  if constexpr ((MODE & MODE_KIND) == MODE_GENERAL_MAT) in.pix = da.w;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  load_one<P, NQ, T>(in, d, pb, pio, it, r);
  solve_one<P, NQ, T, mode_pivots(MODE), (MODE & MODE_FIX) != 0>(in, d, pb, pio, lds, r, slot,
                                                                                     status);
}

// Largest work-group of the direction-resident schedule for a variant, chosen
// so that the kernel's registers fit without spilling (a 1024-thread group
// leaves 128 VGPRs per lane, 512 leaves 256).
template <int P, int NQ, typename T, int MODE>
constexpr int dir_block_max() {
  if ((MODE & MODE_KIND) == MODE_AFFINE_NOPIVOT) {
    if (sizeof(T) == 8) return P <= 3 ? 512 : 256;
    return P <= 2 ? 1024 : 512;
  }
  if (sizeof(T) == 8) return 512;
  if (MODE & MODE_FIX) return 512;  // the fixup variant needs more than 128 registers
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
template <int P, int NQ, typename T, int MODE>
__global__ void __launch_bounds__((dir_block_max<P, NQ, T, MODE>()))
k_sweep_dir(const int2 *__restrict__ tasks, const KProb *__restrict__ probs,
            const KIO *__restrict__ io, const T *__restrict__ tables, int it,
            const int *__restrict__ stop, int *__restrict__ status) {
  using S = Shape<P, NQ>;
  using LD = Lds<P, NQ, MODE>;
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
  int *lo = reinterpret_cast<int *>(lds + LD::TAB + (size_t)slots * LD::AREA);
  stage_tables<P, NQ, T, MODE>(tables, lds);
  const int32_t *lo_g = pb.level_off + (size_t)g * (pb.n_levels + 1);
  for (int i = threadIdx.x; i <= nl; i += blockDim.x) lo[i] = lo_g[i];
  __syncthreads();
  const int2 *dsc = pb.desc_ef + (size_t)g * pb.ne;
  const int4 *dnb = pb.desc_nb + (size_t)g * pb.ne;
  const int lane = threadIdx.x & 63;
  const int r = lane & (S::SLOT - 1);
  const int slot = (threadIdx.x >> 6) * S::SPW + lane / S::SLOT;

  auto fetch = [&](InputsOf<P, NQ, T, MODE> &in, int L, int t) {
    in.valid = L < nl && t < lo[L + 1];
    in.e = 0;
    in.flags = 0;
    in.nb[0] = in.nb[1] = in.nb[2] = in.nb[3] = -1;
    if (in.valid) {
      const int2 ef = dsc[t];
      const int4 nb = dnb[t];
      in.e = ef.x;
      in.flags = ef.y;
      if constexpr (mode_pivots(MODE))  // this direction's pivoting bit
        in.flags |= (int)((pb.mask[(size_t)d * pb.ne + ef.x] >> 7) << 12);
      in.nb[0] = nb.x;
      in.nb[1] = nb.y;
      in.nb[2] = nb.z;
      in.nb[3] = nb.w;
    }
    load_one<P, NQ, T>(in, d, pb, pio, it, r);
  };

  InputsOf<P, NQ, T, MODE> cur, nxt;
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
    solve_one<P, NQ, T, mode_pivots(MODE), (MODE & MODE_FIX) != 0>(cur, d, pb, pio, lds, r,
                                                                                       slot, status);
    if (L2 != L) __syncthreads();  // the level's fluxes are upwind values of the next
    cur = nxt;
    L = L2;
    base = base2;
  }
}

// ---------------------------------------------------------------------------
// Wave-pipelined thread-per-solve schedule (affine elements, p <= 2,
// pivot-free).  One work-group per (problem, direction) with W waves.  The
// 64-element chunks of the upwind levels, in level order, are dealt
// round-robin to the waves; lane l of a chunk solves one element.  The local
// matrix and its LU factors do not depend on upwind data, so a wave assembles
// and factors its next chunk while earlier levels are still being solved;
// only "read the upwind traces, finish the right-hand side, two triangular
// solves, write" waits for the levels below.  Chunks hand off through an LDS
// counter of completed chunks; face traces go through an LDS ring of R levels
// indexed by (level mod R, position in level, face).  An upwind element more
// than R - 1 levels back is read from the angular flux in global memory,
// written before its chunk's counter update.  Waits are bounded by a spin
// count: on expiry the wave sets the status word and every wave leaves the
// kernel.
// ---------------------------------------------------------------------------

constexpr int kPipeMaxWaves = 8;
constexpr int kPipeRing = 4;  // default ring depth (levels)

// Waves per work-group of a pipelined variant (every variant fits in 256
// registers per lane, two waves per SIMD).
template <int P, typename T>
constexpr int pipe_max_waves() {
  return kPipeMaxWaves;
}

// GEN: straight-sided bilinear elements.  The face terms are those of the
// affine case (n ds is constant along a straight edge of a bilinear map, so a
// face contributes (Omega . N_f) times the 1D face mass); the volume terms
// and the source are summed over the quadrature points with the element's
// geometry there (tables_g: V, Dxi, Deta at the points).  Only the prep
// differs; the critical part is the affine one.
template <int P, int NQ, typename T, bool FIX, bool GEN>
__global__ void __launch_bounds__((pipe_max_waves<P, T>() * 64))
k_sweep_pipe(const int2 *__restrict__ tasks, const KProb *__restrict__ probs,
             const KIO *__restrict__ io, const T *__restrict__ tables, const T *__restrict__ tables_g, int it,
             const int *__restrict__ stop, int *__restrict__ status, int ring_levels, int ring_width,
             int global_sync, long long wait_spins) {
  using S = Shape<P, NQ>;
  constexpr int P1 = S::P1, N = S::N, Q = S::Q;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  if (*stop) return;
  const int W = blockDim.x >> 6;
  const int2 tk = tasks[blockIdx.x];
  const int prob = tk.x, d = tk.y;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  const int g = pb.dir_group[d];
  const int nl = pb.n_levels_g[g];
  const int ne = pb.ne;
  T *ring = lds + S::TAB_A;  // [R][4][P1][ring_width]: position fastest (no bank conflicts)
  int *lo = reinterpret_cast<int *>(ring + (size_t)ring_levels * ring_width * 4 * P1);
  int *done = lo + nl + 1;   // chunks completed
  int *abort_flag = done + 1;
  for (int i = threadIdx.x; i < S::TAB_A; i += blockDim.x) lds[i] = tables[i];
  const int32_t *lo_g = pb.level_off + (size_t)g * (pb.n_levels + 1);
  for (int i = threadIdx.x; i <= nl; i += blockDim.x) lo[i] = lo_g[i];
  if (threadIdx.x == 0) {
    *done = 0;
    *abort_flag = 0;
  }
  __syncthreads();  // the only work-group barrier

  const VEF_GLOBAL int *dsc = gmem(reinterpret_cast<const int *>(pb.desc_ef + (size_t)g * ne));
  const VEF_GLOBAL int *dnb = gmem(reinterpret_cast<const int *>(pb.desc_nb + (size_t)g * ne));
  const VEF_GLOBAL uint32_t *dup = gmem(pb.desc_up + (size_t)g * ne * 4);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const T ox = static_cast<T>(pb.omega[2 * d]);
  const T oy = static_cast<T>(pb.omega[2 * d + 1]);
  const VEF_GLOBAL double *phi = gmem(it == 0 ? pio.phi_in : pio.mom);
  const VEF_GLOBAL double *q_iso = gmem(pio.q_iso);
  VEF_GLOBAL T *psi = gmem(static_cast<T *>(pio.psi));
  const VEF_GLOBAL double *sig = gmem(pb.sig);

  // Tasks are the 64-element chunks of the levels in level order; wave w
  // takes tasks w, w + W, ...  `before` counts the tasks of the levels below
  // L: the task may start its critical part once that many have completed.
  int L = 0, base = lo[0], before = 0;
  auto advance = [&](int k) {
    for (int i = 0; i < k && L < nl; ++i) {
      base += 64;
      if (base >= lo[L + 1]) {
        before += (lo[L + 1] - lo[L] + 63) >> 6;
        ++L;
        base = L < nl ? lo[L] : 0;
      }
    }
  };
  // 1D factors of the reference matrices (uniform: scalar loads, held in
  // scalar registers): m = 1D mass, gd = 1D derivative-times-value table.
  // M = m (x) m, Gx = gd (x) m, Gy = m (x) gd with the test index first, and
  // M1 (the face mass) = m.
  const VEF_CONST T *tabc = (const VEF_CONST T *)tables;
  T m1[P1 * P1], gd[P1 * P1];
#pragma unroll
  for (int k = 0; k < P1 * P1; ++k) {
    m1[k] = tabc[S::A_M1 + k];
    gd[k] = tabc[S::A_GD1 + k];
  }
  advance(wave);
  for (; L < nl; advance(W)) {
    const int beg = lo[L], end = lo[L + 1];
    {
      const int t = base + lane;
      const bool valid = t < end;
      // The table reads are loop invariant; an opaque offset keeps the
      // compiler from hoisting all of them (hundreds of values) out of the
      // loop, which would not fit in registers.
      // q_dir and inflow-data tables stay in LDS (paths taken only with
      // those inputs); the opaque offset keeps their reads in the loop.
      int toff = 0;
      asm volatile("" : "+v"(toff));
      const T *WV = lds + S::A_WV + toff;
      const T *WL = lds + S::A_WL + toff;
      // ---- prep: everything that does not depend on upwind values
      int e = 0, flags = 0;
      int nb[4] = {-1, -1, -1, -1};
      uint32_t up[4] = {0u, 0u, 0u, 0u};
      if (valid) {
        e = dsc[2 * t];
        flags = dsc[2 * t + 1];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          nb[f] = dnb[4 * t + f];
          up[f] = dup[4 * t + f];
        }
      }
      T gv[13];
      if constexpr (!GEN) {
        const VEF_GLOBAL T *ga = gmem(static_cast<const T *>(pb.geo_a) + (size_t)e * 16);
#pragma unroll
        for (int k = 0; k < 13; ++k) gv[k] = ga[k];
      } else {
#pragma unroll
        for (int k = 0; k < 13; ++k) gv[k] = T(0);
      }
      const T st = static_cast<T>(sig[2 * e]);
      const T ss = static_cast<T>(sig[2 * e + 1] * kInv4Pi);
      // nodal source s_j = sigma_s / (4 pi) phi_j + q_j.  One branch per
      // array and all N loads of an array issued together (a branch inside
      // the node loop would make every load a separate round trip).
      double pv[N], qv[N];
      if (phi) {
#pragma unroll
        for (int j = 0; j < N; ++j) pv[j] = phi[(size_t)e * N + j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) pv[j] = 0.0;
      }
      if (q_iso) {
#pragma unroll
        for (int j = 0; j < N; ++j) qv[j] = q_iso[(size_t)e * N + j];
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j) qv[j] = 0.0;
      }
      T sj[N];
#pragma unroll
      for (int j = 0; j < N; ++j) sj[j] = ss * static_cast<T>(pv[j]) + static_cast<T>(qv[j]);
      T on[4];
      T b[N];
      T stJ = T(0), gx = T(0), gy = T(0);
      T A[N][N];
      if constexpr (!GEN) {
        const T J = gv[0];
        stJ = st * J;
        gx = gv[1] * ox + gv[2] * oy;
        gy = gv[3] * ox + gv[4] * oy;
#pragma unroll
        for (int f = 0; f < 4; ++f) on[f] = ox * gv[5 + 2 * f] + oy * gv[6 + 2 * f];
        // Right-hand side first: every branch of the prep happens while only
        // these N values are live, the matrix below is straight-line code.
        // b = J (m (x) m) s by sum factorisation: node (a, b) = a + P1 * b.
        {
          T h[P1][P1];  // h[a][d] = sum_c m[a][c] s[c][d]
#pragma unroll
          for (int a = 0; a < P1; ++a)
#pragma unroll
            for (int dd = 0; dd < P1; ++dd) {
              T acc = T(0);
#pragma unroll
              for (int c = 0; c < P1; ++c) acc += m1[a * P1 + c] * sj[c + P1 * dd];
              h[a][dd] = acc;
            }
#pragma unroll
          for (int a = 0; a < P1; ++a)
#pragma unroll
            for (int bb = 0; bb < P1; ++bb) {
              T acc = T(0);
#pragma unroll
              for (int dd = 0; dd < P1; ++dd) acc += m1[bb * P1 + dd] * h[a][dd];
              b[a + P1 * bb] = J * acc;
            }
        }
        if (pio.q_dir) {
          const VEF_GLOBAL double *qd = gmem(pio.q_dir + ((size_t)d * ne + e) * Q);
          T qv[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) qv[q] = static_cast<T>(qd[q]);
#pragma unroll
          for (int i = 0; i < N; ++i) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += WV[q * N + i] * qv[q];
            b[i] += J * acc;
          }
        }
      } else {
        // Omega . N_f: n ds is constant along the edge and the face weights sum to one
        const VEF_GLOBAL T *gfq = gmem(static_cast<const T *>(pb.geo_f) + (size_t)e * 8 * NQ);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          T acc = T(0);
#pragma unroll
          for (int q = 0; q < NQ; ++q) acc += ox * gfq[(f * NQ + q) * 2] + oy * gfq[(f * NQ + q) * 2 + 1];
          on[f] = acc;
        }
        const VEF_GLOBAL T *gq = gmem(static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5);
        const VEF_CONST T *tg = (const VEF_CONST T *)tables_g;  // V, Dxi, Deta [Q][N]
        const VEF_GLOBAL double *qdp = pio.q_dir ? gmem(pio.q_dir + ((size_t)d * ne + e) * Q) : nullptr;
#pragma unroll
        for (int i = 0; i < N; ++i) b[i] = T(0);
        // b_i = sum_q wJ_q V_qi (sum_j V_qj s_j + q_dir,q)
#pragma unroll 1
        for (int q = 0; q < Q; ++q) {
          const T wJ = gq[5 * q];
          T src = qdp ? static_cast<T>(qdp[q]) : T(0);
#pragma unroll
          for (int j = 0; j < N; ++j) src += tg[q * N + j] * sj[j];
          src *= wJ;
#pragma unroll
          for (int i = 0; i < N; ++i) b[i] += tg[q * N + i] * src;
        }
      }
      if (pio.psi_bc) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          if (!(valid && ((flags >> f) & 1) && nb[f] < 0)) continue;
          const VEF_GLOBAL double *bc = gmem(pio.psi_bc + ((size_t)d * pb.nbf + (-nb[f] - 1)) * NQ);
          T bq[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) bq[q] = static_cast<T>(bc[q]);
#pragma unroll
          for (int a = 0; a < P1; ++a) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc += WL[q * P1 + a] * bq[q];
            b[face_node<P>(f, a)] -= on[f] * acc;
          }
        }
      }
      // Matrix: reference matrices scaled by the element's constants, plus
      // on * M1 on the outflow faces (a select, not a branch: a divergent
      // branch around the update would copy the whole matrix).
      T cf[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) cf[f] = ((flags >> f) & 1) ? T(0) : on[f];
      // A[(a,b)][(c,d)] = stJ m_ac m_bd - gx gd_ac m_bd - gy m_ac gd_bd
      //                  = m_bd X_ac - gd_bd Y_ac
      if constexpr (!GEN) {
        T X[P1 * P1], Y[P1 * P1];
#pragma unroll
        for (int k = 0; k < P1 * P1; ++k) {
          X[k] = stJ * m1[k] - gx * gd[k];
          Y[k] = gy * m1[k];
        }
#pragma unroll
        for (int bb = 0; bb < P1; ++bb)
#pragma unroll
          for (int a = 0; a < P1; ++a)
#pragma unroll
            for (int dd = 0; dd < P1; ++dd)
#pragma unroll
              for (int c = 0; c < P1; ++c)
                A[a + P1 * bb][c + P1 * dd] = m1[bb * P1 + dd] * X[a * P1 + c] - gd[bb * P1 + dd] * Y[a * P1 + c];
      } else {
        // A_ij = sum_q (sigma_t wJ_q V_qi - (adj(F)_q Omega) . grad V_qi) V_qj
        const VEF_GLOBAL T *gq = gmem(static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5);
        const VEF_CONST T *tg = (const VEF_CONST T *)tables_g;
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
          for (int j = 0; j < N; ++j) A[i][j] = T(0);
#pragma unroll 1
        for (int q = 0; q < Q; ++q) {
          const T wJ = gq[5 * q], a00 = gq[5 * q + 1], a01 = gq[5 * q + 2], a10 = gq[5 * q + 3],
                  a11 = gq[5 * q + 4];
          const T sw = st * wJ, gxq = a00 * ox + a01 * oy, gyq = a10 * ox + a11 * oy;
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const T ci = sw * tg[q * N + i] - (gxq * tg[(Q + q) * N + i] + gyq * tg[(2 * Q + q) * N + i]);
#pragma unroll
            for (int j = 0; j < N; ++j) A[i][j] += ci * tg[q * N + j];
          }
        }
      }
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int a = 0; a < P1; ++a)
#pragma unroll
          for (int c = 0; c < P1; ++c) A[face_node<P>(f, a)][face_node<P>(f, c)] += cf[f] * m1[a * P1 + c];
      // LU factors in place (natural order), reciprocal pivots kept
      T inv[N];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        inv[k] = recip(A[k][k]);
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
          A[i][k] *= inv[k];
#pragma unroll
          for (int j = k + 1; j < N; ++j) A[i][j] -= A[i][k] * A[k][j];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      // Keep the factorisation ahead of the wait: without these register
      // dependencies the compiler may sink the arithmetic past the wait loop
      // (it has no memory effects), which would put it on the critical path.
#pragma unroll
      for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) asm volatile("" : "+v"(A[i][j]));
        asm volatile("" : "+v"(inv[i]));
        asm volatile("" : "+v"(b[i]));
      }

      // ---- wait for every task of the levels below L
      if (L > 0) {
        long long spins = 0;
        while (__hip_atomic_load(done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < before) {
          if (++spins > wait_spins) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lane == 0) atomicOr(status, 2);
            return;
          }
          if ((spins & 63) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
          __builtin_amdgcn_s_sleep(1);
        }
      }

      // ---- critical: upwind traces, substitution, outputs.  The wave runs
      // it at raised issue priority: the other waves of its SIMD are doing
      // their (long, independent) prep, which would otherwise take every
      // second issue slot of this dependent chain.
      __builtin_amdgcn_s_setprio(3);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (!valid || !((flags >> f) & 1) || nb[f] < 0) continue;
        const uint32_t u = up[f];
        const int gap = (int)(u & 255u);
        const int pos_up = (int)((u >> 8) & 0x3FFFFFu);
        const int f_up = (int)(u >> 30);
        T tr[P1];
        if (gap < ring_levels) {
          const T *src = ring + (size_t)((L - gap) & (ring_levels - 1)) * 4 * P1 * ring_width + pos_up;
#pragma unroll
          for (int c = 0; c < P1; ++c) tr[c] = src[(size_t)(f_up * P1 + P - c) * ring_width];
        } else {
          const VEF_GLOBAL T *src = psi + ((size_t)d * ne + nb[f]) * N;
#pragma unroll
          for (int c = 0; c < P1; ++c) tr[c] = src[face_node<P>(f_up, P - c)];
        }
#pragma unroll
        for (int a = 0; a < P1; ++a) {
          T acc = T(0);
#pragma unroll
          for (int c = 0; c < P1; ++c) acc += m1[a * P1 + c] * tr[c];
          b[face_node<P>(f, a)] -= on[f] * acc;
        }
      }
      // forward (unit lower) and backward substitution
#pragma unroll
      for (int i = 1; i < N; ++i)
#pragma unroll
        for (int k = 0; k < i; ++k) b[i] -= A[i][k] * b[k];
#pragma unroll
      for (int i = N - 1; i >= 0; --i) {
#pragma unroll
        for (int j = i + 1; j < N; ++j) b[i] -= A[i][j] * b[j];
        b[i] *= inv[i];
      }
      if constexpr (FIX) {  // negative-flux fixup (see zero_and_scale_slot), one element per lane
        bool neg = false;
#pragma unroll
        for (int i = 0; i < N; ++i) neg |= b[i] < T(0);
        if (neg) {
          // balance weight of node (a, b): sigma_t times the integral of its
          // basis function (affine: J sm_a sm_b, sm = row sums of m; bilinear:
          // the quadrature sum with wJ at each point) plus (Omega . N_f) sm_pos
          // for each outflow face f through it
          const T ste = static_cast<T>(sig[2 * e]);
          T stJ = T(0);
          if constexpr (!GEN) stJ = ste * gmem(static_cast<const T *>(pb.geo_a))[(size_t)e * 16];
          T cx = T(0), cp = T(0);
          for (int i = 0; i < N; ++i) {
            const int a = i % P1, bb = i / P1;
            T cw;
            if constexpr (GEN) {
              const VEF_GLOBAL T *gq = gmem(static_cast<const T *>(pb.geo_v) + (size_t)e * Q * 5);
              const VEF_CONST T *tg = (const VEF_CONST T *)tables_g;
              T cv = T(0);
              for (int q = 0; q < Q; ++q) cv += gq[5 * q] * tg[q * N + i];
              cw = ste * cv;
            } else {
              T sa = T(0), sb = T(0);
              for (int c = 0; c < P1; ++c) {
                sa += m1[a * P1 + c];
                sb += m1[bb * P1 + c];
              }
              cw = stJ * sa * sb;
            }
            for (int f = 0; f < 4; ++f) {
              const bool on_face = (f == 0) ? (bb == 0) : (f == 1) ? (a == P) : (f == 2) ? (bb == P) : (a == 0);
              if (!on_face || ((flags >> f) & 1)) continue;
              const int pos = (f == 0) ? a : (f == 1) ? bb : (f == 2) ? (P - a) : (P - bb);
              T sp = T(0);
              for (int c = 0; c < P1; ++c) sp += m1[pos * P1 + c];
              cw += on[f] * sp;
            }
            cx += cw * b[i];
            if (b[i] > T(0)) cp += cw * b[i];
          }
          const T alpha = (cx > T(0) && cp > T(0)) ? cx / cp : T(0);
#pragma unroll
          for (int i = 0; i < N; ++i) b[i] = b[i] > T(0) ? alpha * b[i] : T(0);
        }
      }
      // outflow traces for the levels below
      if (valid) {
        T *dst = ring + (size_t)(L & (ring_levels - 1)) * 4 * P1 * ring_width + (t - beg);
#pragma unroll
        for (int f = 0; f < 4; ++f)
          if (!((flags >> f) & 1))
#pragma unroll
            for (int c = 0; c < P1; ++c) dst[(size_t)(f * P1 + c) * ring_width] = b[face_node<P>(f, c)];
      }
      VEF_GLOBAL T *out = psi + ((size_t)d * ne + e) * N;
      if (global_sync) {  // some consumer reads fluxes from global memory: store before publishing
        if (valid) {
#pragma unroll
          for (int i = 0; i < N; ++i) out[i] = b[i];
        }
        __builtin_amdgcn_s_waitcnt(0);  // vmcnt, expcnt, lgkmcnt all zero
      }
      // ---- chunk complete: publish.  Chunks of level L + 1 cannot finish
      // before every chunk of level L, so the count of completed chunks
      // reaches `before` exactly when the levels below L are complete.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) __hip_atomic_fetch_add(done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_s_setprio(0);
      // the angular flux, off the critical path when only LDS hands off
      if (valid) {
        bool bad = false;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          if (!global_sync) out[i] = b[i];
          bad |= !__builtin_isfinite(b[i]);  // a class test: "x - x != 0" may be contracted
        }
        if (bad) atomicOr(status, 1);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row-set LU for affine elements of degree 3 and 4 (pivot-free, as the other
// affine kernels: straight faces and sigma_t > 0).  A slot is one 16-lane DPP
// row; lane l holds RS rows of the augmented system [A | b], row l + s H of
// set s (RS = 1, H = 16 for p = 3; RS = 2, H = 13 for p = 4).  Step K of the
// right-looking elimination broadcasts pivot row K from its lane with
// row_newbcast fused into the multiply-add (v_fmac_*_dpp), so an update costs
// one instruction and no lane moves; rows of the mixed set below the pivot
// take the multipliers, the other sets' rows are all below it (or all above,
// and skip the step).  The pivot entry and the multipliers of the mixed set
// are cleared as they are used, and the reciprocal pivots are kept, so the
// back substitution is the same broadcast update on the right-hand side
// column.  Work per slot: n^2 (n + 3)/3 fused updates for p = 4 spread over
// 13 lanes (2/3 n^3 flops for LU plus 2 n^2 for the substitutions).
// ---------------------------------------------------------------------------

template <int P>
struct LuShape {
  static constexpr int P1 = P + 1, N = P1 * P1;
  static constexpr int SLOT = 16, SPW = 4;
  static constexpr int RS = (N + SLOT - 1) / SLOT;  // rows held per lane
  static constexpr int H = (N + RS - 1) / RS;       // lanes holding rows
};

template <int P, int NQ, bool CLS = false>
struct LuLds {
  static constexpr int P1 = P + 1, N = P1 * P1, Q = NQ * NQ;
  // tables: 1D mass m [P1][P1], 1D derivative table gd [P1][P1], boundary
  // table w_q l_a(s_q) [NQ][P1]
  static constexpr int T_M = 0, T_GD = P1 * P1, T_WL = 2 * P1 * P1, TAB = 2 * P1 * P1 + NQ * P1;
  // per slot: geometry [16] (J, adj(F), face chords), nodal source [N], q_dir [Q],
  // upwind traces or boundary data of the four faces [4][TW] (streaming kernel)
  static constexpr int TW = P1 > NQ ? P1 : NQ;
  static constexpr int A_G = 0, A_S = 16, A_QD = 16 + N, A_TR = 16 + N + Q, A_SC = A_TR + 4 * TW;
  // class matrices (CLS): traces of interior faces in A_TR, boundary data in
  // A_TB [4][TW], each zero where the face has the other kind or is outflow
  static constexpr int A_TB = A_SC + 4;
  static constexpr int AREA = CLS ? ((A_TB + 4 * TW + 1) / 2) * 2
                                  : ((A_SC + 3 + 1) / 2) * 2;  // A_SC: sigma_t, Omega_x, Omega_y
};

// Columns of a class matrix K = A^-1 R (shared local matrices, p >= 3): the
// solution of every solve of the class is K times its staged inputs, in the
// order of the slot's area: nodal source [N] (R = J M), interior traces
// [4][TW] (R = the inflow face terms with m), boundary data [4][TW] (with
// w l), q_dir [Q] (R = J (w V)^T).  Stored T [NCOL][16][RS] per class, entry
// [j][r][s] = K[r + s H][j].
template <int P, int NQ>
struct ClsCols {
  static constexpr int P1 = P + 1, N = P1 * P1, Q = NQ * NQ, TW = P1 > NQ ? P1 : NQ;
  static constexpr int C_S = 0, C_FI = N, C_FB = N + 4 * TW, C_QD = N + 8 * TW, NCOL = N + 8 * TW + Q;
  static constexpr int RS = (N + 15) / 16;
  static constexpr int BLOCK = NCOL * 16 * RS;
};

// Per-lane inputs of one solve (loaded ahead of it).
template <int P, int NQ, typename T>
struct SolveInL {
  static constexpr int Q = NQ * NQ, QD = (Q + 15) / 16;
  int e, flags;
  int nb[4];
  bool valid;
  T g;      // geometry value r of the element (16 per element)
  T s[2];   // nodal source at nodes r and r + 16
  T qd[QD]; // q_dir at volume points r, r + 16, ...
};

template <int P, int NQ, typename T>
__device__ __forceinline__ void load_one(SolveInL<P, NQ, T> &in, int d, const KProb &pb, const KIO &pio, int it,
                                         int r) {
#pragma clang fp contract(off)  // the same rounding as the streaming kernel's staging
  constexpr int N = LuShape<P>::N, Q = NQ * NQ;
  const int e = in.e;
  if (!in.valid) return;
  in.g = static_cast<const T *>(pb.geo_a)[(size_t)e * 16 + r];
  const double *phi = it == 0 ? pio.phi_in : pio.mom;
  const double ss = pb.sig[2 * e + 1] * kInv4Pi;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int node = r + 16 * k;
    T sv = T(0);
    if (node < N) {
      if (phi) sv = static_cast<T>(ss) * static_cast<T>(phi[(size_t)e * N + node]);
      if (pio.q_iso) sv += static_cast<T>(pio.q_iso[(size_t)e * N + node]);
    }
    in.s[k] = sv;
  }
#pragma unroll
  for (int k = 0; k < SolveInL<P, NQ, T>::QD; ++k) {
    const int q = r + 16 * k;
    in.qd[k] = (pio.q_dir && q < Q) ? static_cast<T>(pio.q_dir[((size_t)d * pb.ne + e) * Q + q]) : T(0);
  }
}

// One block of class-matrix columns [cb, cb + L) against the slot's own
// area entries [ab, ab + L).
template <int L, int RS, typename T>
__device__ __forceinline__ void cls_block_own(T (&x)[RS], const T *K, const T *area, int cb, int ab) {
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const T in = area[ab + l];
#pragma unroll
    for (int s = 0; s < RS; ++s) x[s] += gload(K + (size_t)(cb + l) * 16 * RS + s) * in;
  }
}

// One block of class-matrix columns [cb, cb + L) against area entries
// [ab, ab + L) of the wave's four slots: slot q takes the columns q, q + 4,
// ... and adds its share to the sums acc[t] of every slot t.
template <int L, int RS, int AREA, typename T>
__device__ __forceinline__ void cls_block_split(T (&acc)[4][RS], const T *K, const T *area, int cb, int ab, int q) {
#pragma unroll
  for (int ll = 0; ll < (L + 3) / 4; ++ll) {
    const int l = q + 4 * ll;
    const int lc = l < L ? l : L - 1;
    T kv[RS];
    if constexpr (RS == 2) {
      typedef T V2 __attribute__((ext_vector_type(2)));
      const V2 v = gload(reinterpret_cast<const V2 *>(K + (size_t)(cb + lc) * 16 * RS));
      kv[0] = v.x;
      kv[1] = v.y;
    } else {
#pragma unroll
      for (int s = 0; s < RS; ++s) kv[s] = gload(K + (size_t)(cb + lc) * 16 * RS + s);
    }
#pragma unroll
    for (int s = 0; s < RS; ++s) kv[s] = l < L ? kv[s] : T(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T in = area[(t - q) * AREA + ab + lc];
#pragma unroll
      for (int s = 0; s < RS; ++s) acc[t][s] += kv[s] * in;
    }
  }
}

// x = K in for the solve's class matrix K (ClsCols) and its inputs staged in
// the slot's area (LuLds<P, NQ, true>); rows r + s H of lane r.  When the
// wave's four slots solve systems of one class (the usual case: a level's
// solves are listed direction by direction) the columns are shared out over
// the slots and a reduction across them completes each slot's sums; else
// each slot multiplies by its own class's matrix.  Blocks of boundary data
// and q_dir are skipped when the run has none.
template <int P, int NQ, typename T>
__device__ __forceinline__ void cls_product(T (&x)[LuShape<P>::RS], const KProb &pb, const KIO &pio, const T *area,
                                            bool valid, int cls, int r) {
  using C = ClsCols<P, NQ>;
  using LD = LuLds<P, NQ, true>;
  constexpr int RS = LuShape<P>::RS, TW = C::TW;
  const int q = (threadIdx.x & 63) >> 4;
  const bool bc = pio.psi_bc != nullptr, qd = pio.q_dir != nullptr;
  const int cl = valid ? cls : -1;
  int c0 = __builtin_amdgcn_readfirstlane(cl);
  c0 = c0 < 0 ? 0 : c0;
  const bool same = __builtin_amdgcn_ballot_w64(cl >= 0 && cl != c0) == 0;
  const T *K = static_cast<const T *>(pb.cls_inv) + r * RS;
  if (same) {
    K += (size_t)c0 * C::BLOCK;
    T acc[4][RS];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int s = 0; s < RS; ++s) acc[t][s] = T(0);
    cls_block_split<C::N, RS, LD::AREA>(acc, K, area, C::C_S, LD::A_S, q);
    cls_block_split<4 * TW, RS, LD::AREA>(acc, K, area, C::C_FI, LD::A_TR, q);
    if (bc) cls_block_split<4 * TW, RS, LD::AREA>(acc, K, area, C::C_FB, LD::A_TB, q);
    if (qd) cls_block_split<C::Q, RS, LD::AREA>(acc, K, area, C::C_QD, LD::A_QD, q);
    // reduce-scatter over the slots: slot q keeps the sums of its own
    // inputs, exchanging with slot q ^ 1 (lanes 16 apart), then q ^ 2 (32)
    const bool o1 = (q & 1) != 0, o2 = (q & 2) != 0;
    T h[2][RS];
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const T keep = o1 ? acc[2 * tt + 1][s] : acc[2 * tt][s];
        const T give = o1 ? acc[2 * tt][s] : acc[2 * tt + 1][s];
        h[tt][s] = keep + __shfl_xor(give, 16);
      }
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const T keep = o2 ? h[1][s] : h[0][s];
      const T give = o2 ? h[0][s] : h[1][s];
      x[s] = keep + __shfl_xor(give, 32);
    }
  } else {
    K += (size_t)(cls < 0 ? 0 : cls) * C::BLOCK;
#pragma unroll
    for (int s = 0; s < RS; ++s) x[s] = T(0);
    cls_block_own<C::N, RS>(x, K, area, C::C_S, LD::A_S);
    cls_block_own<4 * TW, RS>(x, K, area, C::C_FI, LD::A_TR);
    if (bc) cls_block_own<4 * TW, RS>(x, K, area, C::C_FB, LD::A_TB);
    if (qd) cls_block_own<C::Q, RS>(x, K, area, C::C_QD, LD::A_QD);
  }
}

// Row rr = node (a, b) of an affine element's local matrix (test index
// first), without the right-hand side: A[(a,b)][(c,d)] = m_bd (stJ m_ac -
// gx gd_ac) - gd_bd (gy m_ac), plus (Omega . N_f) m_{pos,c} at face node c of
// each outflow face f (bit f of inflow clear) through (a, b), pos the node's
// position on that face.  m, gd: the 1D mass and derivative tables.
template <int P, typename T>
__device__ __forceinline__ void affine_lu_row(T *row, int rr, const T *m1, const T *gdt, T stJ, T gx, T gy,
                                              const T (&on)[4], unsigned inflow) {
  constexpr int P1 = P + 1;
  const int a = rr % P1, b = rr / P1;
  T Xa[P1], Ya[P1], mb[P1], gb[P1];
#pragma unroll
  for (int c = 0; c < P1; ++c) {
    const T mac = m1[a * P1 + c];
    Xa[c] = stJ * mac - gx * gdt[a * P1 + c];
    Ya[c] = gy * mac;
    mb[c] = m1[b * P1 + c];
    gb[c] = gdt[b * P1 + c];
  }
#pragma unroll
  for (int dd = 0; dd < P1; ++dd)
#pragma unroll
    for (int c = 0; c < P1; ++c) row[c + P1 * dd] = mb[dd] * Xa[c] - gb[dd] * Ya[c];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    if ((inflow >> f) & 1u) continue;
    // outflow face: a multiply by zero off the face instead of a branch
    const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
    const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
    const T cf = on_face ? on[f] : T(0);
#pragma unroll
    for (int c = 0; c < P1; ++c) row[face_node<P>(f, c)] += cf * m1[pos * P1 + c];
  }
}

// Assemble and solve one element-direction system from the slot's staged
// geometry and sources (all 16 lanes of the slot call it).  CLS: the solve's
// local matrix is shared by its class (index cls) and the handle holds the
// classes' inverses (pb.cls_inv); only the right-hand side is assembled.  tab: the LDS
// tables (LuLds), wv: w V [Q][n] in global memory (direction-dependent source
// only), area: the slot's LDS area.  The upwind traces of the inflow faces
// (face node c of face f, in the face order of the downwind element) are
// read from the angular flux here (SRC_LDS false; boundary data then from
// pio.psi_bc) or come from the area's trace buffer, which also holds the
// inflow data of boundary faces (SRC_LDS true).
template <int P, int NQ, typename T, bool FIX, bool COH, bool SRC_LDS, bool CLS = false>
__device__ __forceinline__ void lu_core(int e, int d, bool valid, int flags, const int (&nb)[4], T ox, T oy, T st,
                                        const KProb &pb, const KIO &pio, const T *tab, const T *wv, T *area, int r,
                                        int *status, int cls = 0) {
  using S = LuShape<P>;
  using LD = LuLds<P, NQ>;
  constexpr int P1 = S::P1, N = S::N, RS = S::RS, H = S::H, Q = NQ * NQ;
  const T *m1 = tab + LD::T_M;
  const T *gdt = tab + LD::T_GD;
  const T *WL = tab + LD::T_WL;
  const int ne = pb.ne;
  const unsigned mask = valid ? (unsigned)flags & 15u : 0u;
  T tr[4][P1];
  if constexpr (!SRC_LDS) {
    // every lane reads them all
    const T *psi = static_cast<const T *>(pio.psi);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
      for (int c = 0; c < P1; ++c) tr[f][c] = T(0);
      if (valid && ((mask >> f) & 1u) && nb[f] >= 0) {
        const int f2 = (flags >> (4 + 2 * f)) & 3;
        const T *up = psi + ((size_t)d * ne + nb[f]) * N;
#pragma unroll
        for (int c = 0; c < P1; ++c) tr[f][c] = ld_psi<COH>(up + face_node<P>(f2, P - c));
      }
    }
  }
  const T *g = area + LD::A_G;
  const T J = g[0];
  const T stJ = st * J;
  const T gx = g[1] * ox + g[2] * oy;
  const T gy = g[3] * ox + g[4] * oy;
  T on[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) on[f] = ox * g[5 + 2 * f] + oy * g[6 + 2 * f];

  // assembly of the lane's rows, right-hand side first (the traces are dead
  // before the matrix is live): b = J (m (x) m) s + J (w V)^T q_dir - the
  // inflow face terms; A[(a,b)][(c,d)] = m_bd (stJ m_ac - gx gd_ac)
  // - gd_bd (gy m_ac) (test index first), plus (Omega . N_f) m on the
  // outflow faces.  With class matrices (CLS) none of this: the solution is
  // the class matrix times the staged inputs.
  T A[RS][N + 1];
#pragma unroll
  for (int s = 0; s < RS && !CLS; ++s) {
    const int row = r + s * H;
    const bool row_ok = valid && r < H && row < N;
    const int rr = (r < H && row < N) ? row : N - 1;
    const int a = rr % P1, b = rr / P1;
    T rhs = T(0);
#pragma unroll
    for (int dd = 0; dd < P1; ++dd) {
      T acc = T(0);
#pragma unroll
      for (int c = 0; c < P1; ++c) acc += m1[a * P1 + c] * area[LD::A_S + c + P1 * dd];
      rhs += m1[b * P1 + dd] * acc;
    }
    rhs *= J;
    if (pio.q_dir) {
      T acc = T(0);
      for (int q = 0; q < Q; ++q) acc += wv[q * N + rr] * area[LD::A_QD + q];
      rhs += J * acc;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
      const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
      if (!(((mask >> f) & 1u) && row_ok && on_face)) continue;
      T acc = T(0);
      const T *trl = area + LD::A_TR + f * LD::TW;
      if (nb[f] >= 0) {
#pragma unroll
        for (int c = 0; c < P1; ++c) {
          if constexpr (SRC_LDS)
            acc += m1[pos * P1 + c] * trl[c];
          else
            acc += m1[pos * P1 + c] * tr[f][c];
        }
      } else if (pio.psi_bc) {
        const double *bc = pio.psi_bc + ((size_t)d * pb.nbf + (-nb[f] - 1)) * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if constexpr (SRC_LDS)
            acc += WL[q * P1 + pos] * trl[q];
          else
            acc += WL[q * P1 + pos] * static_cast<T>(bc[q]);
        }
      }
      rhs -= on[f] * acc;
    }
    A[s][N] = rhs;
  }
  T x[RS];
  if constexpr (CLS) {
    cls_product<P, NQ, T>(x, pb, pio, area, valid, cls, r);
  } else {
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int row = r + s * H;
      const int rr = (r < H && row < N) ? row : N - 1;
      affine_lu_row<P, T>(A[s], rr, m1, gdt, stJ, gx, gy, on, mask);
    }
    T idg[RS];
    lu_rows<N, RS, H, T>(A, idg, r);
#pragma unroll
    for (int s = 0; s < RS; ++s) x[s] = A[s][N] * idg[s];
  }

  if constexpr (FIX) {
    // negative-flux fixup (see zero_and_scale_slot) over the slot's rows:
    // balance weight of node (a, b) = stJ sm_a sm_b + outflow faces through
    // it (Omega . N_f) sm_pos, sm = row sums of m
    bool neg = false;
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int row = r + s * H;
      neg |= valid && r < H && row < N && x[s] < T(0);
    }
    if (__builtin_amdgcn_ballot_w64(neg) != 0) {
      T cx = T(0), cp = T(0);
      int nneg = 0;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int row = r + s * H;
        const bool row_ok = valid && r < H && row < N;
        const int rr = row_ok ? row : 0;
        const int a = rr % P1, b = rr / P1;
        T sa = T(0), sb = T(0);
        for (int c = 0; c < P1; ++c) {
          sa += m1[a * P1 + c];
          sb += m1[b * P1 + c];
        }
        T c0 = stJ * sa * sb;
        for (int f = 0; f < 4; ++f) {
          const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
          if (!on_face || ((mask >> f) & 1u)) continue;
          const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
          T sp = T(0);
          for (int c = 0; c < P1; ++c) sp += m1[pos * P1 + c];
          c0 += on[f] * sp;
        }
        if (row_ok) {
          cx += c0 * x[s];
          if (x[s] > T(0)) cp += c0 * x[s];
          nneg += x[s] < T(0) ? 1 : 0;
        }
      }
#pragma unroll
      for (int m = 1; m < 16; m <<= 1) {
        cx += __shfl_xor(cx, m);
        cp += __shfl_xor(cp, m);
        nneg += __shfl_xor(nneg, m);
      }
      if (nneg > 0) {
        const T alpha = (cx > T(0) && cp > T(0)) ? cx / cp : T(0);
#pragma unroll
        for (int s = 0; s < RS; ++s) x[s] = x[s] > T(0) ? alpha * x[s] : T(0);
      }
    }
  }
  T *out = static_cast<T *>(pio.psi) + ((size_t)d * ne + e) * N;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int row = r + s * H;
    if (valid && r < H && row < N) {
      st_psi<COH>(out + row, x[s]);
      if (!__builtin_isfinite(x[s])) atomicOr(status, 1);  // non-finite unknown
    }
  }
}

// One solve from its loaded inputs: stage them in the slot's LDS area, read
// the upwind traces (every lane reads them all), assemble and solve.
template <int P, int NQ, typename T, bool FIX, bool COH = false>
__device__ __forceinline__ void solve_one_lu(const SolveInL<P, NQ, T> &in, int d, const KProb &pb, const KIO &pio,
                                             const T *tab, const T *wv, T *area, int r, int *status) {
  using LD = LuLds<P, NQ>;
  constexpr int P1 = P + 1, N = P1 * P1, Q = NQ * NQ;
  const int e = in.e;
  const bool valid = in.valid;

  // staging (wave-local)
  area[LD::A_G + r] = in.g;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (r + 16 * k < N) area[LD::A_S + r + 16 * k] = in.s[k];
  if (pio.q_dir) {
#pragma unroll
    for (int k = 0; k < SolveInL<P, NQ, T>::QD; ++k)
      if (r + 16 * k < Q) area[LD::A_QD + r + 16 * k] = in.qd[k];
  }
  wave_sync_lds();
  const T ox = static_cast<T>(pb.omega[2 * d]);
  const T oy = static_cast<T>(pb.omega[2 * d + 1]);
  const T st = static_cast<T>(pb.sig[2 * (valid ? e : 0)]);
  lu_core<P, NQ, T, FIX, COH, false>(e, d, valid, in.flags, in.nb, ox, oy, st, pb, pio, tab, wv, area, r, status);
}

// Stage the LU tables (m, gd, w l) from the affine table blob into LDS.
template <int P, int NQ, typename T>
__device__ __forceinline__ void stage_tables_lu(const T *__restrict__ tables, T *lds) {
  using S = Shape<P, NQ>;
  using LD = LuLds<P, NQ>;
  constexpr int PP = S::P1 * S::P1;
  for (int i = threadIdx.x; i < LD::TAB; i += blockDim.x) {
    T v;
    if (i < PP)
      v = tables[S::A_M1 + i];
    else if (i < 2 * PP)
      v = tables[S::A_GD1 + i - PP];
    else
      v = tables[S::A_WL + i - 2 * PP];
    lds[i] = v;
  }
}

// Level-synchronous schedule with the row-set LU (one slot per solve).
template <int P, int NQ, typename T, bool FIX>
__global__ void __launch_bounds__(256)
k_sweep_level_lu(const int4 *__restrict__ desc, int n_solves, const KProb *__restrict__ probs,
                 const KIO *__restrict__ io, const T *__restrict__ tables, int it, const int *__restrict__ stop,
                 int *__restrict__ status) {
  using S = LuShape<P>;
  using LD = LuLds<P, NQ>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int slot = (threadIdx.x >> 6) * S::SPW + (lane >> 4);
  const int sid = xcd_block(blockIdx.x, gridDim.x) * ((blockDim.x >> 6) * S::SPW) + slot;
  SolveInL<P, NQ, T> in;
  in.valid = sid < n_solves;
  int4 da = make_int4(0, 0, 0, 0), db = make_int4(-1, -1, -1, -1);
  if (in.valid) {
    da = desc[2 * (size_t)sid];
    db = desc[2 * (size_t)sid + 1];
  }
  if (*stop) return;
  stage_tables_lu<P, NQ, T>(tables, lds);
  __syncthreads();
  in.e = da.x;
  const int d = da.y & 0xffff, prob = da.y >> 16;
  in.flags = da.z & 0xffff;
  in.nb[0] = db.x;
  in.nb[1] = db.y;
  in.nb[2] = db.z;
  in.nb[3] = db.w;
  const KProb &pb = probs[prob];
  const KIO &pio = io[prob];
  load_one<P, NQ, T>(in, d, pb, pio, it, r);
  solve_one_lu<P, NQ, T, FIX>(in, d, pb, pio, lds, tables + Shape<P, NQ>::A_WV, lds + LD::TAB + (size_t)slot * LD::AREA,
                              r, status);
}

// Level-synchronous schedule, streaming form (handles of one problem): a
// launch of at most the resident work-groups, each slot taking the level's
// solves sid, sid + S, ... (S slots in the grid, at most 16 solves a slot).
// The 16 lanes of a slot load the descriptors of the slot's solves at the
// start (lane k those of its k-th solve); the inputs of the next solve,
// upwind traces included (written by earlier launches), are loaded while the
// current one is factored, so the chain of dependent loads is paid once per
// launch and not once per solve.
template <int P, int NQ, typename T>
struct LuPre {
  static constexpr int TW = LuLds<P, NQ>::TW, NT = (4 * TW + 15) / 16;
  // raw loaded values: every lane issues the same loads on every solve (an
  // unused one reads a valid dummy address), and nothing is computed from a
  // load until the solve is staged, so that no wait for them comes before the
  // current solve's work
  T g, sc;               // sc: sigma_t (lane 0), Omega_x (lane 1), Omega_y (lane 2)
  T tr[NT];              // upwind trace values
  double bc[sizeof(T) == sizeof(double) ? 1 : NT];  // boundary inflow data (double precision: in tr)
  double phi[2], qi[2];  // scalar flux and isotropic source at nodes r, r + 16
  double ss;             // sigma_s
  int use;               // bit k: tr[k] used, bit 8 + k: bc[k] used, bit 16: phi present
};

template <int P, int NQ, typename T>
__device__ __forceinline__ void lu_prefetch(LuPre<P, NQ, T> &x, int e, int d, int flags, const int (&nb)[4],
                                            bool valid, const KProb &pb, const KIO &pio, int it, int r) {
  using X = LuPre<P, NQ, T>;
  constexpr int P1 = P + 1, N = P1 * P1, TW = X::TW;
  constexpr bool kWide = sizeof(T) == sizeof(double);  // boundary data and traces share one load
  if (!valid) {
    e = 0;
    d = 0;
    flags = 0;
  }
  const double *dummy = pb.sig;
  x.g = gload(static_cast<const T *>(pb.geo_a) + (size_t)e * 16 + r);
  x.sc = static_cast<T>(gload(r == 0 ? pb.sig + 2 * e : pb.omega + 2 * d + (r == 2 ? 1 : 0)));
  x.ss = gload(pb.sig + 2 * e + 1);
  const double *phi = it == 0 ? pio.phi_in : pio.mom;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int node = r + 16 * k < N ? r + 16 * k : 0;
    x.phi[k] = gload(phi ? phi + (size_t)e * N + node : dummy);
    x.qi[k] = gload(pio.q_iso ? pio.q_iso + (size_t)e * N + node : dummy);
  }
  // trace entry i = f TW + c: upwind value at face node c, or inflow data at
  // quadrature point c of a boundary face
  const T *psi = static_cast<const T *>(pio.psi);
  int use = 0;
#pragma unroll
  for (int k = 0; k < X::NT; ++k) {
    const int i = r + 16 * k;
    const int f = (i < 4 * TW ? i : 0) / TW, c = (i < 4 * TW ? i : 0) - f * TW;
    const int u = f == 0 ? nb[0] : f == 1 ? nb[1] : f == 2 ? nb[2] : nb[3];
    const bool inflow = i < 4 * TW && ((flags >> f) & 1);
    const bool up = inflow && u >= 0 && c < P1;
    const bool bnd = inflow && u < 0 && pio.psi_bc && c < NQ;
    const int f2 = (flags >> (4 + 2 * f)) & 3;
    const T *pa = up ? psi + ((size_t)d * pb.ne + u) * N + face_node_sel<P>(f2, P - c) : static_cast<const T *>(pb.geo_a);
    const double *pbnd = bnd ? pio.psi_bc + ((size_t)d * pb.nbf + (-u - 1)) * NQ + c : dummy;
    if constexpr (kWide) {
      x.tr[k] = gload(bnd ? reinterpret_cast<const T *>(pbnd) : pa);
    } else {
      x.tr[k] = gload(pa);
      x.bc[k] = gload(pbnd);
    }
    use |= (up || (kWide && bnd) ? 1 : 0) << k;
    use |= (bnd ? 1 : 0) << (8 + k);
  }
  use |= (phi ? 1 : 0) << 16;
  x.use = valid ? use : 0;
}

// Stage a prefetched solve in the slot's area; the direction-dependent
// source q_dir (not prefetched) is read here.  CLS: the area of the class
// matrices, boundary data apart from the traces.
template <int P, int NQ, typename T, bool CLS = false>
__device__ __forceinline__ void lu_stage(const LuPre<P, NQ, T> &x, T *area, const KProb &pb, const KIO &pio, int e,
                                         int d, bool valid, int r) {
#pragma clang fp contract(off)
  using X = LuPre<P, NQ, T>;
  using LD = LuLds<P, NQ, CLS>;
  constexpr int N = (P + 1) * (P + 1), Q = NQ * NQ;
  constexpr bool kWide = sizeof(T) == sizeof(double);
  area[LD::A_G + r] = x.g;
  // nodal source sigma_s / (4 pi) phi + q_iso, rounded as in load_one
  const double ss = x.ss * kInv4Pi;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (r + 16 * k < N) {
      T sv = T(0);
      if ((x.use >> 16) & 1) sv = static_cast<T>(ss) * static_cast<T>(x.phi[k]);
      if (pio.q_iso) sv += static_cast<T>(x.qi[k]);
      area[LD::A_S + r + 16 * k] = valid ? sv : T(0);
    }
  if (pio.q_dir) {
#pragma unroll
    for (int k = 0; k < (Q + 15) / 16; ++k) {
      const int q = r + 16 * k;
      if (q < Q) area[LD::A_QD + q] = valid ? static_cast<T>(gload(pio.q_dir + ((size_t)d * pb.ne + e) * Q + q)) : T(0);
    }
  }
#pragma unroll
  for (int k = 0; k < X::NT; ++k)
    if (r + 16 * k < 4 * X::TW) {
      T v = T(0);
      if ((x.use >> k) & 1) v = x.tr[k];  // (double precision: boundary data as well)
      if constexpr (!kWide) {
        if ((x.use >> (8 + k)) & 1) v = static_cast<T>(x.bc[k]);
      }
      if constexpr (CLS) {
        const bool bnd = (x.use >> (8 + k)) & 1;
        area[LD::A_TR + r + 16 * k] = bnd ? T(0) : v;
        area[LD::A_TB + r + 16 * k] = bnd ? v : T(0);
      } else {
        area[LD::A_TR + r + 16 * k] = v;
      }
    }
  if (r < 3) area[LD::A_SC + r] = x.sc;
}

constexpr int kLuStreamMax = 16;  // solves per slot and launch (one per lane of the slot)

template <int P, int NQ, typename T, bool FIX, bool CLS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CLS ? (sizeof(T) == 4 ? 4 : 3) : sizeof(T) == 4 ? 3 : 2)))
k_sweep_level_lus(const int4 *__restrict__ desc, int n_solves, const KProb *__restrict__ probs,
                  const KIO *__restrict__ io, const T *__restrict__ tables, int it, const int *__restrict__ stop,
                  int *__restrict__ status) {
  using S = LuShape<P>;
  using LD = LuLds<P, NQ, CLS>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int slot = (threadIdx.x >> 6) * S::SPW + (lane >> 4);
  const int per_block = (blockDim.x >> 6) * S::SPW;
  const int n_slots = gridDim.x * per_block;
  // Slot s of work-group b takes the solves b per_block + s + k n_slots
  // (plain block order: the XCD-aware order halves the HBM reads of the
  // element data of the row-set LU but measured slower on the 512x512 p = 4
  // sweep).  With class matrices (CLS) the solves are cut into kXcds
  // contiguous ranges, one per XCD (work-groups go to the XCDs round robin;
  // the host makes the grid a multiple of kXcds), taken in the same strided
  // order within the range: a level's solves are listed direction by
  // direction, so each XCD's L2 holds the matrices of about an eighth of the
  // classes.  The host sizes the grid so that no slot has more than
  // kLuStreamMax solves.
  int sid0, stride, lim;
  if constexpr (CLS) {
    const int nxb = gridDim.x / kXcds, x = blockIdx.x % kXcds;
    const int chunk = (n_solves + kXcds - 1) / kXcds;
    const int lo = x * chunk;
    lim = lo + chunk < n_solves ? lo + chunk : n_solves;
    sid0 = lo + (blockIdx.x / kXcds) * per_block + slot;
    stride = nxb * per_block;
  } else {
    sid0 = blockIdx.x * per_block + slot;
    stride = n_slots;
    lim = n_solves;
  }
  const int sidw = sid0 - (lane >> 4);  // first slot of the wave
  const int n_it = sidw < lim ? (lim - sidw + stride - 1) / stride : 0;
  const KProb &pb = probs[0];
  const KIO &pio = io[0];

  // descriptors of the slot's solves, in LDS after the slot areas: lane k
  // writes those of the slot's k-th solve (element, direction, flags, class;
  // neighbours; flags: inflow faces, neighbour faces << 4, pivoting bit 12,
  // boundary faces << 16), loaded before the stop flag is read
  int *dtab = reinterpret_cast<int *>(lds + LD::TAB + (size_t)per_block * LD::AREA) + slot * (kLuStreamMax * 8);
  int4 da = make_int4(0, 0, 0, 0), db = make_int4(-1, -1, -1, -1);
  {
    const long long sid = (long long)sid0 + (long long)r * stride;
    if (sid < lim) {
      da = desc[2 * sid];
      db = desc[2 * sid + 1];
    }
  }
  if (*stop) return;
  stage_tables_lu<P, NQ, T>(tables, lds);
  {
    int4 *w = reinterpret_cast<int4 *>(dtab + r * 8);
    w[0] = make_int4(da.x, da.y & 0xffff, da.z, CLS ? da.w : 0);
    w[1] = db;
  }
  __syncthreads();
  T *area = lds + LD::TAB + (size_t)slot * LD::AREA;
  const T *wv = tables + Shape<P, NQ>::A_WV;
  LuPre<P, NQ, T> nx;
  auto prefetch = [&](int k) __attribute__((always_inline)) {
    const int4 a = reinterpret_cast<const int4 *>(dtab + k * 8)[0];
    const int4 b = reinterpret_cast<const int4 *>(dtab + k * 8)[1];
    const int nb[4] = {b.x, b.y, b.z, b.w};
    lu_prefetch<P, NQ, T>(nx, a.x, a.y, a.z, nb, (long long)sid0 + (long long)k * stride < lim, pb, pio, it, r);
  };
  prefetch(0);
  for (int k = 0; k < n_it; ++k) {
    const int4 a = reinterpret_cast<const int4 *>(dtab + k * 8)[0];
    const int e = a.x, d = a.y, fl = a.z;
    const bool valid = (long long)sid0 + (long long)k * stride < lim;
    wave_sync_lds();  // the previous solve is done with the area
    lu_stage<P, NQ, T, CLS>(nx, area, pb, pio, e, d, valid, r);
    wave_sync_lds();
    if (k + 1 < n_it) prefetch(k + 1);
    // only the sign of a neighbour index is used by the solve
    const int nb[4] = {(fl >> 16) & 1 ? -1 : 0, (fl >> 17) & 1 ? -1 : 0, (fl >> 18) & 1 ? -1 : 0,
                       (fl >> 19) & 1 ? -1 : 0};
    lu_core<P, NQ, T, FIX, false, true, CLS>(e, d, valid, fl, nb, area[LD::A_SC + 1], area[LD::A_SC + 2],
                                             area[LD::A_SC], pb, pio, lds, wv, area, r, status, a.w);
  }
}

// Class matrix K = A^-1 R (ClsCols) of one class of solves that share their
// local matrix A (one work-group of kClsThreads threads per class, see
// ClassInvLaunch): thread i < n assembles row i of A and of R in double from
// the representative element's geometry, sigma_t and the direction, as the
// row-set LU assembles A and b; then Gauss-Jordan elimination with partial
// pivoting on [A | R] in LDS.  R maps the staged inputs to b: J M for the
// nodal source, -(Omega . N_f) m (interior traces) or -(Omega . N_f) w l
// (boundary data) on the rows of each inflow face f, J (w V)^T for q_dir.
constexpr int kClsThreads = 256;
template <int P, int NQ, typename T>
__global__ void __launch_bounds__(kClsThreads)
k_class_inv(const int4 *__restrict__ rep, const KProb *__restrict__ probs, const T *__restrict__ tables,
            T *__restrict__ out, int *__restrict__ status) {
  using S = LuShape<P>;
  using C = ClsCols<P, NQ>;
  using SH = Shape<P, NQ>;
  constexpr int P1 = S::P1, N = S::N, RS = S::RS, H = S::H, Q = C::Q, TW = C::TW;
  constexpr int W = N + C::NCOL;
  __shared__ double m1[P1 * P1], gd[P1 * P1], wl[NQ * P1];
  __shared__ double M[N][W + 1];
  __shared__ double fac[N];
  __shared__ int piv;
  const int t = threadIdx.x;
  const int4 rp = rep[blockIdx.x];
  const KProb &pb = probs[0];
  for (int i = t; i < P1 * P1; i += kClsThreads) {
    m1[i] = static_cast<double>(tables[SH::A_M1 + i]);
    gd[i] = static_cast<double>(tables[SH::A_GD1 + i]);
  }
  for (int i = t; i < NQ * P1; i += kClsThreads) wl[i] = static_cast<double>(tables[SH::A_WL + i]);
  for (int x = t; x < N * W; x += kClsThreads) M[x / W][x % W] = 0.0;
  __syncthreads();
  if (t < N) {
    const T *g = static_cast<const T *>(pb.geo_a) + (size_t)rp.x * 16;
    const double ox = pb.omega[2 * rp.y], oy = pb.omega[2 * rp.y + 1];
    const double J = static_cast<double>(g[0]);
    const double stJ = pb.sig[2 * rp.x] * J;
    const double gx = static_cast<double>(g[1]) * ox + static_cast<double>(g[2]) * oy;
    const double gy = static_cast<double>(g[3]) * ox + static_cast<double>(g[4]) * oy;
    const unsigned inflow = (unsigned)rp.z & 15u;
    double on[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) on[f] = ox * static_cast<double>(g[5 + 2 * f]) + oy * static_cast<double>(g[6 + 2 * f]);
    double row[N];
    affine_lu_row<P, double>(row, t, m1, gd, stJ, gx, gy, on, inflow);
    for (int j = 0; j < N; ++j) M[t][j] = row[j];
    const int a = t % P1, b = t / P1;
    double *R = &M[t][N];
    for (int dd = 0; dd < P1; ++dd)
      for (int c = 0; c < P1; ++c) R[C::C_S + c + P1 * dd] = J * m1[a * P1 + c] * m1[b * P1 + dd];
    for (int f = 0; f < 4; ++f) {
      const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
      if (!((inflow >> f) & 1u) || !on_face) continue;
      const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
      for (int c = 0; c < P1; ++c) R[C::C_FI + f * TW + c] = -on[f] * m1[pos * P1 + c];
      for (int qq = 0; qq < NQ; ++qq) R[C::C_FB + f * TW + qq] = -on[f] * wl[qq * P1 + pos];
    }
    const T *wv = tables + SH::A_WV;
    for (int qq = 0; qq < Q; ++qq) R[C::C_QD + qq] = J * static_cast<double>(wv[qq * N + t]);
  }
  __syncthreads();
  for (int k = 0; k < N; ++k) {
    if (t == 0) {
      int pr = k;
      double best = fabs(M[k][k]);
      for (int i = k + 1; i < N; ++i)
        if (fabs(M[i][k]) > best) {
          best = fabs(M[i][k]);
          pr = i;
        }
      piv = pr;
      if (best == 0.0) atomicOr(status, 1);
    }
    __syncthreads();
    const int pr = piv;
    if (pr != k)
      for (int j = t; j < W; j += kClsThreads) {
        const double v = M[k][j];
        M[k][j] = M[pr][j];
        M[pr][j] = v;
      }
    __syncthreads();
    const double pk = M[k][k];
    if (t < N) fac[t] = t == k ? 0.0 : M[t][k] / pk;
    __syncthreads();
    for (int x = t; x < N * W; x += kClsThreads) {
      const int i = x / W, j = x - i * W;
      if (i != k) M[i][j] -= fac[i] * M[k][j];
    }
    __syncthreads();
    for (int j = t; j < W; j += kClsThreads) M[k][j] /= pk;
    __syncthreads();
  }
  T *o = out + (size_t)blockIdx.x * C::BLOCK;
  for (int x = t; x < C::BLOCK; x += kClsThreads) {
    const int j = x / (16 * RS), r = (x / RS) % 16, s = x % RS;
    const int row = r + s * H;
    o[x] = (r < H && row < N) ? static_cast<T>(M[row][N + j]) : T(0);
  }
}

template <int P, int NQ, typename T>
hipError_t launch_class_inv_t(const ClassInvLaunch &C) {
  if constexpr (P < 3) {
    return hipErrorInvalidValue;
  } else {
    if (C.n_cls <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_class_inv<P, NQ, T>), dim3(C.n_cls), dim3(kClsThreads), 0, C.stream, C.rep, C.probs,
                       static_cast<const T *>(C.tables), static_cast<T *>(C.out), C.status);
    return hipGetLastError();
  }
}

// Row order of partial pivoting for each local matrix of a general element
// (element matrices, p = 3) that is not certified for elimination in natural
// order.  A 16-lane slot per listed (element, direction): lane r forms row r
// of A from the element matrices with the sums of the sweep's assembly, then
// the slot runs Gauss-Jordan elimination with partial pivoting; the lane
// whose row is the pivot of step k writes out[16 i + k] = r.  Elimination in
// natural order of the rows taken in that order meets the pivots of partial
// pivoting, so the sweep needs no pivot search (nor its divergent path).
// Every step picks a lane not yet used (a zero pivot too), so each out row is
// a permutation of 0..15.
template <int P, typename T>
__global__ void __launch_bounds__(256)
k_pivot_order(const int2 *__restrict__ list, int n, const KProb *__restrict__ probs, int prob,
              uint8_t *__restrict__ out) {
  using EM = EMat<P>;
  constexpr int P1 = P + 1, N = P1 * P1, W = 16 / sizeof(T);
  static_assert(N == 16, "element matrices: degree 3");
  __shared__ T pv[16][N + 1];
  const int r = threadIdx.x & 15, slot = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + slot;
  const KProb &pb = probs[prob];
  T A[N];
#pragma unroll
  for (int j = 0; j < N; ++j) A[j] = j == r ? T(1) : T(0);  // past the list: identity
  if (i < n) {
    const int e = list[i].x, d = list[i].y;
    const T *em = static_cast<const T *>(pb.emat) + (size_t)e * EM::SIZE;
    const unsigned mask = pb.mask[(size_t)d * pb.ne + e] & 15u;
    const T ox = static_cast<T>(pb.omega[2 * d]), oy = static_cast<T>(pb.omega[2 * d + 1]);
    const T st = static_cast<T>(pb.sig[2 * e]);
    const int a = r % P1, b = r / P1;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int at = ((j / W) * 16 + r) * W + j % W;
      A[j] = st * em[at] - (ox * em[EM::OFF_GX + at] + oy * em[EM::OFF_GY + at]);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const bool on_face = (f == 0) ? (b == 0) : (f == 1) ? (a == P) : (f == 2) ? (b == P) : (a == 0);
      const int pos = (f == 0) ? a : (f == 1) ? b : (f == 2) ? (P - a) : (P - b);
      if (!on_face || ((mask >> f) & 1u)) continue;
      const T *fx = em + EM::OFF_F + (2 * f) * P1 * P1 + pos * P1, *fy = fx + P1 * P1;
#pragma unroll
      for (int c = 0; c < P1; ++c) A[face_node<P>(f, c)] += ox * fx[c] + oy * fy[c];
    }
  }
  T rhs = T(0);
  bool active = true;
  int my_k = r;
  gj_pivot<16, N, 0, T>(A, rhs, r, active, my_k, &pv[slot][0]);
  if (i < n) out[(size_t)i * 16 + my_k] = (uint8_t)r;
}

template <int P, typename T>
hipError_t launch_pivot_order_t(const PivotOrderLaunch &L) {
  if (L.n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pivot_order<P, T>), dim3((L.n + 15) / 16), dim3(256), 0, L.stream, L.list, L.n, L.probs,
                     L.prob, L.out);
  return hipGetLastError();
}

// Direction-resident schedule with the row-set LU (as k_sweep_dir).
template <int P, int NQ, typename T, bool FIX>
__global__ void __launch_bounds__(256)
k_sweep_dir_lu(const int2 *__restrict__ tasks, const KProb *__restrict__ probs, const KIO *__restrict__ io,
               const T *__restrict__ tables, int it, const int *__restrict__ stop, int *__restrict__ status) {
  using S = LuShape<P>;
  using LD = LuLds<P, NQ>;
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
  int *lo = reinterpret_cast<int *>(lds + LD::TAB + (size_t)slots * LD::AREA);
  stage_tables_lu<P, NQ, T>(tables, lds);
  const int32_t *lo_g = pb.level_off + (size_t)g * (pb.n_levels + 1);
  for (int i = threadIdx.x; i <= nl; i += blockDim.x) lo[i] = lo_g[i];
  __syncthreads();
  const int2 *dsc = pb.desc_ef + (size_t)g * pb.ne;
  const int4 *dnb = pb.desc_nb + (size_t)g * pb.ne;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15;
  const int slot = (threadIdx.x >> 6) * S::SPW + (lane >> 4);
  T *area = lds + LD::TAB + (size_t)slot * LD::AREA;
  const T *wv = tables + Shape<P, NQ>::A_WV;

  auto fetch = [&](SolveInL<P, NQ, T> &in, int L, int t) {
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
    load_one<P, NQ, T>(in, d, pb, pio, it, r);
  };

  SolveInL<P, NQ, T> cur, nxt;
  int L = 0, base = 0;
  fetch(cur, 0, slot);
  while (L < nl) {
    int L2 = L, base2 = base + slots;
    if (base2 >= lo[L + 1]) {
      L2 = L + 1;
      base2 = L2 < nl ? lo[L2] : 0;
    }
    fetch(nxt, L2, base2 + slot);
    solve_one_lu<P, NQ, T, FIX>(cur, d, pb, pio, lds, wv, area, r, status);
    if (L2 != L) __syncthreads();  // the level's fluxes are upwind values of the next
    cur = nxt;
    L = L2;
    base = base2;
  }
}

template <int P, int NQ, typename T, bool FIX>
hipError_t launch_level_lu_t(const SweepLaunch &L) {
  if constexpr (P < 3) {
    return hipErrorInvalidValue;
  } else {
    using LD = LuLds<P, NQ>;
    const int block = L.block > 256 ? 256 : (L.block < 64 ? 64 : L.block);
    const int per_block = (block / 64) * LuShape<P>::SPW;
    const size_t bytes = sizeof(T) * ((size_t)LD::TAB + (size_t)LD::AREA * per_block);
    if (bytes > L.lds_max) return hipErrorInvalidValue;
    int grid = (L.count + per_block - 1) / per_block;
    if (grid == 0) return hipSuccess;
    if (!L.desc) return hipErrorInvalidValue;
    // + the descriptor tables (the class-matrix form has larger areas)
    const size_t area_s = L.shared ? LuLds<P, NQ, true>::AREA : LD::AREA;
    const size_t bytes_s =
        sizeof(T) * ((size_t)LD::TAB + area_s * per_block) + sizeof(int) * 8 * kLuStreamMax * per_block;
    if (L.single && L.n_cu > 0 && bytes_s <= L.lds_max) {
      // streaming form: the resident work-groups, and enough of them that a
      // slot has at most kLuStreamMax solves
      // resident blocks per CU: a host query, cached per device and block
      // size (a level-synchronous sweep launches once per level)
      static std::atomic<int> cache[64][4][2];
      int dev = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e != hipSuccess) return e;
      if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
      const bool cacheable = block % 64 == 0;
      const int cv = L.shared ? 1 : 0;
      int per_cu = cacheable ? cache[dev][block / 64 - 1][cv].load(std::memory_order_relaxed) : 0;
      if (per_cu == 0) {
        e = L.shared ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_level_lus<P, NQ, T, FIX, true>,
                                                                   block, bytes_s)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_level_lus<P, NQ, T, FIX, false>,
                                                                   block, bytes_s);
        if (e != hipSuccess) return e;
        if (per_cu < 1) return hipErrorInvalidConfiguration;
        if (cacheable) cache[dev][block / 64 - 1][cv].store(per_cu, std::memory_order_relaxed);
      }
      const int cap = per_block * kLuStreamMax;
      const int res = per_cu * L.n_cu;
      if (L.shared) {
        // a multiple of kXcds work-groups, each XCD's covering an eighth of
        // the solves (see k_sweep_level_lus)
        const int per_x = (L.count + kXcds - 1) / kXcds;
        const int need = (per_x + per_block - 1) / per_block, lo_x = (per_x + cap - 1) / cap;
        int gx = res / kXcds;
        if (gx > need) gx = need;
        if (gx < lo_x) gx = lo_x;
        grid = gx * kXcds;
      } else {
        const int lo = (L.count + cap - 1) / cap;
        if (grid > res) grid = res > lo ? res : lo;
      }
      if (L.shared)
        hipLaunchKernelGGL((k_sweep_level_lus<P, NQ, T, FIX, true>), dim3(grid), dim3(block), bytes_s, L.stream,
                           L.desc, L.count, L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
      else
        hipLaunchKernelGGL((k_sweep_level_lus<P, NQ, T, FIX, false>), dim3(grid), dim3(block), bytes_s, L.stream,
                           L.desc, L.count, L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
      return hipGetLastError();
    }
    // the class inverses are used by the streaming form only
    if (L.shared) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep_level_lu<P, NQ, T, FIX>), dim3(grid), dim3(block), bytes, L.stream, L.desc, L.count,
                       L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
    return hipGetLastError();
  }
}

template <int P, int NQ, typename T, bool FIX>
hipError_t launch_dir_lu_t(const SweepLaunch &L) {
  if constexpr (P < 3) {
    return hipErrorInvalidValue;
  } else {
    if (L.count == 0) return hipSuccess;
    using LD = LuLds<P, NQ>;
    int block = ((L.width * 16 + 63) / 64) * 64;
    block = block < 64 ? 64 : (block > 256 ? 256 : block);
    for (; block >= 64; block -= 64) {
      const size_t bytes = sizeof(T) * ((size_t)LD::TAB + (size_t)LD::AREA * (block / 64) * LuShape<P>::SPW) +
                           sizeof(int) * ((size_t)L.max_levels + 1);
      if (bytes <= L.lds_max) {
        hipLaunchKernelGGL((k_sweep_dir_lu<P, NQ, T, FIX>), dim3(L.count), dim3(block), bytes, L.stream, L.list,
                           L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
        return hipGetLastError();
      }
    }
    return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Persistent schedule: one launch per sweep (and kernel variant) with every
// resident wave a worker.  The solves of each (problem, direction class,
// upwind level) are cut into tasks of a few rounds of consecutive solves
// (element-major, all directions of the class); the tasks, sorted by level,
// are dealt round-robin to the workers (wave w takes tasks w, w + W, ...).
// A task waits only for the tasks that hold its upwind elements' solves of
// the same directions (a predecessor list made at create), through one flag
// per task set to the sweep number when the task is done.  A predecessor is
// on a lower level, so it precedes the task in every worker's list, and all
// tasks finish provided every worker is resident: the grid is sized from the
// kernel's occupancy.  The angular flux that crosses work-groups is written
// and read with agent-scope atomic stores and loads, and a task's flag is
// stored once its stores have completed, so no cache-wide fence is needed.
// Waits are bounded: on expiry a wave sets the status word and a global
// abort flag that makes every other wave leave as well.  Each wave loads the
// inputs of its next solves (element data, not the upwind traces) while it
// solves the current ones.
// ---------------------------------------------------------------------------

// Per-variant solve policy: the row-set LU (affine, p >= 3) or the
// row-per-lane kernels (general elements).
template <int P, int NQ, typename T, int MODE, bool LU = ((MODE & MODE_KIND) == MODE_AFFINE_LU)>
struct FlowPolicy;

template <int P, int NQ, typename T, int MODE>
struct FlowPolicy<P, NQ, T, MODE, true> {
  static constexpr int SLOT = 16, SPW = 4;
  // the double-precision rows leave no registers for the next round's inputs
  // (with them the kernel spills; measured slower on the 512x512 p = 4 sweep)
  static constexpr bool kPrefetch = sizeof(T) == 4;
  static constexpr int TAB = LuLds<P, NQ>::TAB, AREA = LuLds<P, NQ>::AREA;
  using In = SolveInL<P, NQ, T>;
  static __device__ __forceinline__ void stage(const T *tables, T *lds) { stage_tables_lu<P, NQ, T>(tables, lds); }
  static __device__ __forceinline__ void solve(const In &in, int d, const KProb &pb, const KIO &pio,
                                               const T *tables, T *lds, int r, int slot, int *status) {
    solve_one_lu<P, NQ, T, false, true>(in, d, pb, pio, lds, tables + Shape<P, NQ>::A_WV,
                                        lds + TAB + (size_t)slot * AREA, r, status);
  }
};

template <int P, int NQ, typename T, int MODE>
struct FlowPolicy<P, NQ, T, MODE, false> {
  static constexpr int SLOT = Shape<P, NQ>::SLOT, SPW = Shape<P, NQ>::SPW;
  static constexpr bool kPrefetch = true;
  static constexpr int TAB = Lds<P, NQ, MODE>::TAB, AREA = Lds<P, NQ, MODE>::AREA;
  using In = InputsOf<P, NQ, T, MODE, true>;  // the level-synchronous kernel's inputs and arithmetic
  static __device__ __forceinline__ void stage(const T *tables, T *lds) { stage_tables<P, NQ, T, MODE>(tables, lds); }
  static __device__ __forceinline__ void solve(const In &in, int d, const KProb &pb, const KIO &pio,
                                               const T *tables, T *lds, int r, int slot, int *status) {
    (void)tables;
    solve_one<P, NQ, T, mode_pivots(MODE), false, true>(in, d, pb, pio, lds, r, slot, status);
  }
};

// One slot's work item: the solve's inputs and its direction and problem.
template <typename In>
struct FlowItem {
  In in;
  int d, prob;
};

template <int P, int NQ, typename T, int MODE>
__global__ void __launch_bounds__(256, 2)
k_sweep_flow(const int4 *__restrict__ desc, const int2 *__restrict__ tasks, int n_tasks,
             const int *__restrict__ pred_ptr, const int *__restrict__ pred_idx, int *__restrict__ flags,
             int own_base, int *__restrict__ abort_flag, const KProb *__restrict__ probs,
             const KIO *__restrict__ io, const T *__restrict__ tables, int it, const int *__restrict__ stop,
             int *__restrict__ status, long long wait_spins) {
  using Pol = FlowPolicy<P, NQ, T, MODE>;
  using Item = FlowItem<typename Pol::In>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *lds = reinterpret_cast<T *>(smem_raw);
  if (*stop) return;
  Pol::stage(tables, lds);
  __syncthreads();  // the only work-group barrier: waves work independently from here on
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int W = gridDim.x * (blockDim.x >> 6);
  const int w = blockIdx.x * (blockDim.x >> 6) + wave;
  const int r = lane & (Pol::SLOT - 1);
  const int sw = lane / Pol::SLOT;         // slot within the wave
  const int slot = wave * Pol::SPW + sw;  // slot within the work-group (LDS area)
  const int epoch = it + 1;               // flag value of a task done in this sweep
  if (w >= n_tasks) return;

  auto fetch = [&](Item &x, const int2 &tk, int rd) {
    // the solve's packed descriptor (element, direction | problem << 16,
    // flags, pivot-order entry; neighbours), as the level kernels read it
    const int k = rd * Pol::SPW + sw;
    x.in.valid = k < tk.y;
    int4 da = make_int4(0, 0, 0, 0), db = make_int4(-1, -1, -1, -1);
    if (x.in.valid) {
      da = desc[2 * ((size_t)tk.x + k)];
      db = desc[2 * ((size_t)tk.x + k) + 1];
    }
    x.in.e = da.x;
    x.d = da.y & 0xffff;
    // a task holds solves of one problem and a wave's slots one task: the
    // problem's records come through the scalar cache
    x.prob = __builtin_amdgcn_readfirstlane(da.y >> 16);
    x.in.flags = da.z & 0xffff;  // inflow faces, neighbour faces, pivoting needed
    x.in.nb[0] = db.x;
    x.in.nb[1] = db.y;
    x.in.nb[2] = db.z;
    x.in.nb[3] = db.w;
    if constexpr ((MODE & MODE_KIND) == MODE_GENERAL_MAT) x.in.pix = da.w;
    load_one<P, NQ, T>(x.in, x.d, probs[x.prob], io[x.prob], it, r);
  };

  int t = w, rd = 0;
  int2 tk = tasks[t];  // (first solve, solves)
  Item cur, nxt;
  if constexpr (Pol::kPrefetch) fetch(cur, tk, 0);
  for (;;) {
    if constexpr (!Pol::kPrefetch) fetch(cur, tk, rd);
    int t2 = t, rd2 = rd + 1;
    int2 tk2 = tk;
    if (rd2 * Pol::SPW >= tk.y) {
      t2 = t + W;
      rd2 = 0;
      if (t2 < n_tasks) tk2 = tasks[t2];
    }
    const bool more = t2 < n_tasks;
    if constexpr (Pol::kPrefetch)
      if (more) fetch(nxt, tk2, rd2);
    if (rd == 0) {
      // the tasks holding this task's upwind fluxes are done in this sweep
      const int q1 = pred_ptr[t + 1];
      for (int q = pred_ptr[t]; q < q1; ++q) {
        const int pt = pred_idx[q];
        long long spins = 0;
        while (__hip_atomic_load(flags + pt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
          if (++spins > wait_spins) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (lane == 0) atomicOr(status, 2);
            return;
          }
          if ((spins & 63) == 0 && __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the trace loads stay after the waits
    }
    Pol::solve(cur.in, cur.d, probs[cur.prob], io[cur.prob], tables, lds, r, slot, status);
    if ((rd + 1) * Pol::SPW >= tk.y) {
      // task complete once this wave's angular-flux stores have completed
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      __builtin_amdgcn_s_waitcnt(0);
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      if (lane == 0) __hip_atomic_store(flags + own_base + t, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!more) break;
    if constexpr (Pol::kPrefetch) cur = nxt;
    t = t2;
    rd = rd2;
    tk = tk2;
  }
}

template <int P, int NQ, typename T, int MODE>
hipError_t launch_flow_t(const SweepLaunch &L) {
  if (L.count == 0) return hipSuccess;
  using Pol = FlowPolicy<P, NQ, T, MODE>;
  constexpr int block = 256;
  const size_t bytes = sizeof(T) * ((size_t)Pol::TAB + (size_t)Pol::AREA * (block / 64) * Pol::SPW);
  if (bytes > L.lds_max) return hipErrorInvalidValue;
  // every worker must be resident: as many work-groups as fit on the device
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sweep_flow<P, NQ, T, MODE>, block, bytes);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int grid = per_cu * L.n_cu;
  const int need = (L.count + (block / 64) - 1) / (block / 64);
  if (grid > need) grid = need;
  if (!L.desc) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_flow<P, NQ, T, MODE>), dim3(grid), dim3(block), bytes, L.stream, L.desc,
                     L.tasks, L.count, L.pred_ptr, L.pred_idx, L.flags, L.own_base, L.abort_flag, L.probs, L.io,
                     static_cast<const T *>(L.tables), L.it, L.stop, L.status, L.wait_spins);
  return hipGetLastError();
}

template <int P, int NQ, typename T, int MODE>
hipError_t launch_dir_t(const SweepLaunch &L);

template <int P, int NQ, typename T, bool FIX, bool GEN>
hipError_t launch_pipe_t(const SweepLaunch &L) {
  if constexpr (P > 2) {
    return hipErrorInvalidValue;
  } else {
    if (L.count == 0) return hipSuccess;
    using S = Shape<P, NQ>;
    // the row-per-lane kernel of the same elements (general ones read the
    // general tables)
    auto rows = [&]() {
      if constexpr (GEN) {
        SweepLaunch G = L;
        G.tables = L.tables_g;
        return launch_dir_t<P, NQ, T, MODE_GENERAL_NOPIVOT | (FIX ? MODE_FIX : 0)>(G);
      } else {
        return launch_dir_t<P, NQ, T, MODE_AFFINE_NOPIVOT | (FIX ? MODE_FIX : 0)>(L);
      }
    };
    {
    constexpr int maxw = pipe_max_waves<P, T>();
    const int waves = L.waves > 0 ? (L.waves > maxw ? maxw : L.waves) : maxw;
    const size_t ring_bytes_per_level = (size_t)L.width * 4 * S::P1 * sizeof(T);
    const size_t fixed = sizeof(T) * S::TAB_A + sizeof(int) * ((size_t)L.max_levels + 3);
    int R = L.ring > 0 ? L.ring : kPipeRing;
    R = R >= 4 ? 4 : (R >= 2 ? 2 : 1);  // a power of two: the slot of a level is a mask
    while (R > 1 && fixed + R * ring_bytes_per_level > L.lds_max) R >>= 1;
    // a level too wide for even one ring slot: the row-per-lane kernel
    if (fixed + R * ring_bytes_per_level > L.lds_max) return rows();
    // lagged couplings (level gap 255) read the previous sweep from global
    // memory and need no store before publishing: max_gap counts only the
    // others
    const int global_sync = (L.max_gap >= R) ? 1 : 0;
    const size_t bytes = fixed + R * ring_bytes_per_level;
    hipLaunchKernelGGL((k_sweep_pipe<P, NQ, T, FIX, GEN>), dim3(L.count), dim3(waves * 64), bytes, L.stream, L.list,
                       L.probs, L.io, static_cast<const T *>(L.tables), static_cast<const T *>(L.tables_g), L.it,
                       L.stop, L.status, R, L.width, global_sync, L.wait_spins);
    return hipGetLastError();
    }
  }
}

// Largest multiple of 64 threads <= want whose LDS fits in lds_max bytes.
template <int P, int NQ, int MODE>
int fit_block(bool fp32, int want, size_t lds_max, int extra_ints, size_t *bytes) {
  using S = Shape<P, NQ>;
  using LD = Lds<P, NQ, MODE>;
  for (int block = want; block >= 64; block -= 64) {
    const int slots = (block / 64) * S::SPW;
    const size_t b = fp32 ? lds_bytes<float>(LD::TAB, LD::AREA, slots, extra_ints)
                          : lds_bytes<double>(LD::TAB, LD::AREA, slots, extra_ints);
    if (b <= lds_max) {
      *bytes = b;
      return block;
    }
  }
  return 0;
}

template <int P, int NQ, typename T, int MODE>
hipError_t launch_level_t(const SweepLaunch &L) {
  size_t bytes = 0;
  const int block = fit_block<P, NQ, MODE>(L.fp32, L.block > 256 ? 256 : L.block, L.lds_max, 0, &bytes);
  if (block == 0) return hipErrorInvalidValue;
  const int per_block = (block / 64) * Shape<P, NQ>::SPW;
  const int grid = (L.count + per_block - 1) / per_block;
  if (grid == 0) return hipSuccess;
  if (!L.desc) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_level<P, NQ, T, MODE>), dim3(grid), dim3(block), bytes, L.stream, L.desc,
                     L.count, L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
  return hipGetLastError();
}

template <int P, int NQ, typename T, int MODE>
hipError_t launch_dir_t(const SweepLaunch &L) {
  if (L.count == 0) return hipSuccess;
  constexpr int SLOT = Shape<P, NQ>::SLOT;
  const int maxb = dir_block_max<P, NQ, T, MODE>();
  int block = ((L.width * SLOT + 63) / 64) * 64;
  block = block < 64 ? 64 : (block > maxb ? maxb : block);
  size_t bytes = 0;
  block = fit_block<P, NQ, MODE>(L.fp32, block, L.lds_max, L.max_levels + 1, &bytes);
  if (block == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_sweep_dir<P, NQ, T, MODE>), dim3(L.count), dim3(block), bytes, L.stream, L.list,
                     L.probs, L.io, static_cast<const T *>(L.tables), L.it, L.stop, L.status);
  return hipGetLastError();
}

template <int P, int NQ, typename T, bool DIR, int FX>
hipError_t launch_mode_fx(const SweepLaunch &L) {
  if (L.flow) {  // persistent schedule: row-per-lane general kernels and the row-set LU, without the fixup
    if constexpr (FX != 0) {
      return hipErrorInvalidValue;
    } else {
      switch (L.mode) {
        case MODE_GENERAL_PIVOT: return launch_flow_t<P, NQ, T, MODE_GENERAL_PIVOT>(L);
        case MODE_GENERAL_NOPIVOT: return launch_flow_t<P, NQ, T, MODE_GENERAL_NOPIVOT>(L);
        case MODE_GENERAL_MAT:
          if constexpr (P == 3) return launch_flow_t<P, NQ, T, MODE_GENERAL_MAT>(L);
          return hipErrorInvalidValue;
        case MODE_AFFINE_LU:
          if constexpr (P >= 3) return launch_flow_t<P, NQ, T, MODE_AFFINE_LU>(L);
          return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (L.mode) {
    case MODE_GENERAL_PIVOT:
      return DIR ? launch_dir_t<P, NQ, T, MODE_GENERAL_PIVOT | FX>(L)
                 : launch_level_t<P, NQ, T, MODE_GENERAL_PIVOT | FX>(L);
    case MODE_GENERAL_NOPIVOT:
      return DIR ? launch_dir_t<P, NQ, T, MODE_GENERAL_NOPIVOT | FX>(L)
                 : launch_level_t<P, NQ, T, MODE_GENERAL_NOPIVOT | FX>(L);
    case MODE_AFFINE_NOPIVOT:
      return DIR ? launch_dir_t<P, NQ, T, MODE_AFFINE_NOPIVOT | FX>(L)
                 : launch_level_t<P, NQ, T, MODE_AFFINE_NOPIVOT | FX>(L);
    case MODE_GENERAL_MAT:
      if constexpr (P == 3)
        return DIR ? launch_dir_t<P, NQ, T, MODE_GENERAL_MAT | FX>(L)
                   : launch_level_t<P, NQ, T, MODE_GENERAL_MAT | FX>(L);
      return hipErrorInvalidValue;
    case MODE_AFFINE_PIPELINE:
      return DIR ? launch_pipe_t<P, NQ, T, FX != 0, false>(L) : hipErrorInvalidValue;
    case MODE_GENERAL_PIPELINE:
      return DIR ? launch_pipe_t<P, NQ, T, FX != 0, true>(L) : hipErrorInvalidValue;
    case MODE_AFFINE_LU:
      return DIR ? launch_dir_lu_t<P, NQ, T, FX != 0>(L) : launch_level_lu_t<P, NQ, T, FX != 0>(L);
    default: return hipErrorInvalidValue;
  }
}

// The fixup is a compile-time variant: kernels without it carry none of its code.
template <int P, int NQ, typename T, bool DIR>
hipError_t launch_mode(const SweepLaunch &L) {
  return L.fixup ? launch_mode_fx<P, NQ, T, DIR, MODE_FIX>(L) : launch_mode_fx<P, NQ, T, DIR, 0>(L);
}

template <int P>
hipError_t launch_class_p(const ClassInvLaunch &C) {
  switch (C.nq - P) {
    case 1: return C.fp32 ? launch_class_inv_t<P, P + 1, float>(C) : launch_class_inv_t<P, P + 1, double>(C);
    case 2: return C.fp32 ? launch_class_inv_t<P, P + 2, float>(C) : launch_class_inv_t<P, P + 2, double>(C);
    case 3: return C.fp32 ? launch_class_inv_t<P, P + 3, float>(C) : launch_class_inv_t<P, P + 3, double>(C);
    default: return hipErrorInvalidValue;
  }
}

template <int P, bool DIR>
hipError_t launch_p(const SweepLaunch &L) {
  switch (L.nq - P) {
    case 1: return L.fp32 ? launch_mode<P, P + 1, float, DIR>(L) : launch_mode<P, P + 1, double, DIR>(L);
    case 2: return L.fp32 ? launch_mode<P, P + 2, float, DIR>(L) : launch_mode<P, P + 2, double, DIR>(L);
    case 3: return L.fp32 ? launch_mode<P, P + 3, float, DIR>(L) : launch_mode<P, P + 3, double, DIR>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

}  // namespace vefk

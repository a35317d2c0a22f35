// Host-side sweep plan: reference tables, geometry at quadrature points, face
// connectivity, per-direction upwind masks, direction classes and upwind
// levels.  Pure C++ (no HIP): everything here runs once at handle creation.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "vef_sweep.h"

namespace vefplan {

constexpr int kMaxP = 4;
constexpr int kMaxM = 3;
constexpr int kMaxDirs = 1024;

// Basis and quadrature tables of one (p, nq) pair, all in double.
struct Tables {
  int p = 0, nq = 0;
  std::vector<double> gl;   // [p+1] Gauss-Lobatto nodes on [0,1], exactly symmetric
  std::vector<double> gx;   // [nq] Gauss-Legendre points on [0,1], exactly symmetric
  std::vector<double> gw;   // [nq] weights, sum 1
  std::vector<double> V;    // [Q][n] basis values at volume points
  std::vector<double> Dx;   // [Q][n] d/dxi
  std::vector<double> Dy;   // [Q][n] d/deta
  std::vector<double> F;    // [nq][p+1] 1D basis at face points
  // affine-element tables: Mhat^T, Ghat_xi^T, Ghat_eta^T [n][n] (entry [j][i]),
  // face mass [p+1][p+1], w V [Q][n], w L [nq][p+1]
  std::vector<double> affine;
};

struct ProblemPlan {
  int p = 0, m = 0, nq = 0, n = 0, Q = 0;
  int ne = 0, nd = 0, nbf = 0;
  // geometry, double precision
  std::vector<double> geo_v;     // [ne][Q][5]: w J, w adjF00, w adjF01, w adjF10, w adjF11
  std::vector<double> geo_f;     // [ne][4][nq][2]: w_s * (n ds) at face points
  std::vector<int32_t> nbr;      // [ne][4]: neighbour element, or -(bf+1) on the boundary
  std::vector<int8_t> nbr_face;  // [ne][4]: neighbour's local face (or -1)
  std::vector<int32_t> bf_ef;    // [nbf]: 4*element + face
  std::vector<uint8_t> mask;     // [nd][ne]: bit f set when face f is inflow
  std::vector<int32_t> dir_group;   // [nd] direction class (identical masks)
  std::vector<int32_t> group_rep;   // [n_groups] first direction of each class
  std::vector<int32_t> level;       // [n_groups][ne] upwind level
  std::vector<int32_t> order;       // [n_groups][ne] elements in (level, id) order
  std::vector<int32_t> level_off;   // [n_groups][n_levels+1] offsets into order
  int n_groups = 0;
  int n_levels = 0;                 // max over classes
  std::vector<int32_t> n_levels_g;  // [n_groups]
  std::vector<int32_t> desc_ef;     // [n_groups][ne][2] in order: element, inflow mask | nbr faces << 4
  std::vector<int32_t> desc_nb;     // [n_groups][ne][4] in order: neighbours
  std::vector<uint32_t> desc_up;    // [n_groups][ne][4] in order, per inflow interior face: level gap
                                    // (bits 0-7, 255 = far), upwind position in its level (8-29),
                                    // upwind local face (30-31); 0 for other faces
  std::vector<uint8_t> lag_mask;    // [n_groups][ne]: bit f set when inflow face f is lagged
  long long n_lagged = 0;           // lagged (direction, element, face) couplings
  long long n_pivoting = 0;         // (direction, element) pairs not certified for natural-order elimination
  int max_gap = 0;                  // largest level gap of an upwind edge that is not lagged
  int max_width = 1;                // widest level over classes
  bool straight = true;             // every face of the mesh is a straight segment
  bool nopivot = false;             // straight faces and sigma_t > 0 everywhere
  bool affine = false;              // every element map is affine (constant J and adj(F))
  bool elem_mat = false;            // solved from precomputed element matrices (set by the handle)
  std::vector<double> geo_a;        // [ne][16] J, adj(F), chords (when affine)
  std::vector<double> omega, weight, sigma_t, sigma_s;
  Tables tab;
};

int build_tables(int p, int nq, Tables &t);

// Tables of the element-local HRT VEF blocks for degree p (1..3) and nq
// Gauss points per direction (p + 2 or p + 3), one blob of doubles:
//   w [Q] tensor weights; vr [Q][nv] the non-zero component of each reference
//   RT_p function (xi-component functions first, node a + (p+2) b, then
//   eta-component functions, node a + (p+1) b); dr [Q][nv][2] its xi and eta
//   derivatives; u [Q][nphi] the Gauss-Legendre nodal phi basis; tv [Q][nt]
//   the transport (Gauss-Lobatto nodal) basis; vrf [4][nq][nv] and
//   tf [4][nq][nt] the same at face points (counter-clockwise parameter);
//   wf [nq] 1D weights.  Q = nq^2.
struct HrtSizes {
  int p = 0, nq = 0, nx = 0, nv = 0, nphi = 0, nt = 0;
  int off_w = 0, off_vr = 0, off_dr = 0, off_u = 0, off_tv = 0, off_vrf = 0, off_tf = 0, off_wf = 0;
  int off_mv = 0, off_dv = 0, off_mu = 0, off_lf = 0, off_lr = 0, total = 0;
};
int hrt_sizes(int p, int nq, HrtSizes &z);
int build_hrt_tables(int p, int nq, std::vector<double> &blob);

// Validates and plans one problem.  lag_cycles: a cyclic upwind graph is
// ordered by releasing elements with lagged couplings instead of failing with
// VEF_ERR_CYCLE.  Returns VEF_OK or a VEF_ERR_* status and a message in err.
// pointwise: the upwind side is chosen at each face quadrature point (a face
// with points of both signs is an inflow face of both of its elements).
int build_problem_plan(const vef_problem_desc &d, bool lag_cycles, bool pointwise, ProblemPlan &out,
                       std::string &err);

}  // namespace vefplan

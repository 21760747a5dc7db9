// Two-centre path (Eq. 1 with capture): data layout and launchers (internal).
//
// A two-centre plan holds one group per (target, projectile) basis pair; the
// paths of a group share sizes, so every launch covers one group.  Each path
// keeps three coupling slots (z, z_mid, z_new of Algorithm 1) holding
//   S  = [[I, K], [K^dag, I]]   column-major [N][N]
//   LU = S factorised with partial pivoting (LAPACK layout, pivots in piv)
//   H  = [[D_T, Q], [L, D_P]]   row-major [N][N]
// Couplings are computed for up to two slots per path in one pass ("jobs":
// job y -> path y / n_sub, slot slot[y % n_sub], position z[y % n_sub]).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace wpccc {

constexpr int kMaxW = 3;          // weights: overlap, target potential, projectile potential
constexpr int kNodeChunk = 32;    // spheroidal nodes per FP64 contraction chunk (8 MFMA k-steps of 4)
constexpr int kTile = 32;         // rows (target) and columns (projectile) per contraction workgroup
// node ranges per contraction tile: the work items of a launch differ in
// their weight count (4 to 12) and node count, so several shorter items per
// tile let the dispatcher balance them over the CUs (partial sums per range
// are added in a fixed order when the blocks are assembled)
constexpr int kContractSplit = 24;
constexpr int kMaxK = 4 * kMaxW;  // weights per (s, t): 2 Bessel orders x (cos, sin) x weights
// coupling slots per path: a step reads three positions (z, z + h/2, z + h);
// a pipelined graph step also forms the next step's last two
constexpr int kSlots2C = 5;
// lane layout of the FP32 16x16x4 MFMA result: 1 if register r of lane l holds
// row 4 (l / 16) + r, 0 if it holds row 4 r + l / 16 (as the FP64 instruction)
constexpr int kF32RowByLaneGroup = 1;

// Per-node fields of one coupling position ([field][n_nodes], SoA):
constexpr int kFCos = 0;          // cos((v z / 2) eta tau)
constexpr int kFSin = 1;          // sin((v z / 2) eta tau)
constexpr int kFW = 2;            // omega W_w, w < kMaxW
constexpr int kFLA = kFW + kMaxW; // five Lagrange weights at r_A
constexpr int kFLB = kFLA + 5;    // five Lagrange weights at r_B
constexpr int kFJ = kFLB + 5;     // J_m(X), m = 0 .. 2L
// then Pbar_l^m(cos theta_A) for l <= LT, m <= l (index l(l+1)/2 + m) from
// field f_pa, and Pbar_l^m(cos theta_B), l <= LP, from field f_pb

// Per-group constants of the two-centre kernels (device copy passed by pointer).
struct Meta2C {
    int LT, LP, L;           // l_max of target, projectile; max of both
    int NT, NP, N;           // states; N = NT + NP
    int nfT, nfP;            // radial functions
    int nrT, nrP;            // grid intervals
    double rmaxT, rmaxP;
    double ZT, ZP;
    int n_eta, n_tau, n_nodes;
    int n_fields;            // f_pb + (LP+1)(LP+2)/2
    int f_pa, f_pb;          // first Legendre field of each side
    int n_w;                 // 2 (overlap, target potential) or 3 (+ projectile potential)
    int q_prior;             // lower-left block: 0 Q^dagger, 1 prior form
    int same;                // one basis object on both centres: blocks s > t from
                             // blocks (t, s) (st_nw, k_2c_assemble)
    int mirror;              // same and the prior form: lower-left block
                             // (-1)^(l_i + l_j) Q_ij, no third weight (k_2c_assemble)
    int mixed;               // 1: contraction products in FP32 (chunk sums promoted to FP64)
    // contraction blocks: rows of block s are the radial functions a >= radT_off[s]
    int radT_off[kMaxL + 2], radP_off[kMaxL + 2];
    int nA[kMaxL + 1], nB[kMaxL + 1];
    int st_off[kMaxL + 1][kMaxL + 1];   // offset of the (s, t) block in tmol
    int n_tmol;                         // doubles of tmol per job
    int stT_off[kMaxL + 2], stP_off[kMaxL + 2];  // state offsets per l
    int n_lT[kMaxL + 1], n_lP[kMaxL + 1];
    int n_tiles;
    int n_split;             // node ranges per contraction tile; tmol holds one partial sum per range
    // interpolated operands: row r of side T is (s, i) with s = block, i < nA[s]
    int rowsT, rowsP;                  // sum_s nA[s], sum_t nB[t]
    int rowT_off[kMaxL + 1], rowP_off[kMaxL + 1];
};

// weights of the (s, t) block: Bessel orders |s-t| and s+t (one if s t = 0),
// each with cos and sin of (v z / 2) eta tau, each with the n_w weights;
// index ((order * 2 + trig) * n_w + w)
__host__ __device__ inline int st_nk(int s, int t, int n_w) { return ((s > 0 && t > 0) ? 2 : 1) * 2 * n_w; }
// weights the contraction forms and stores for block (s, t), in the order
// overlap, target potential, projectile potential.  With one basis on both
// centres (same) exchanging the centres maps block (s, t) to block (t, s)
// transposed, the overlap to itself and the target potential to the
// projectile's (k_2c_assemble): the blocks s < t form all three, the blocks
// s = t the first two, the blocks s > t none.
__host__ __device__ inline int st_nw(int same, int n_w, int s, int t) {
    return same ? (s < t ? 3 : (s == t ? 2 : 0)) : n_w;
}
// The same map takes the overlap of a diagonal block (s, s) at (a, b) to the
// overlap at (b, a), so a tile of such a block above its diagonal (a0 < b0)
// forms the target potential only; k_2c_assemble reads the overlap there
// from the transposed tile.  Contraction tiles: x = s | t << 8 | upper << 16,
// y = a0 | b0 << 16.
constexpr int kTileUpper = 1 << 16;
__host__ __device__ inline bool overlap_mirrored(int same, int s, int t, int a, int b) {
    return same && s == t && a / kTile < b / kTile;
}

struct Jobs {
    int path0;       // first local path of the launch
    int n_sub;       // 1 or 2 coupling positions per path
    int slot[2];
    double z[2];
    // graph replays: z[sub] = zdev[3 * (*step + ahead) + sub] instead
    // (nullptr: z[]); ahead = 1 where a step forms the next step's couplings
    const double* zdev;
    const int* step;
    int ahead;
};

struct NodeArgs {
    const Meta2C* m;
    Jobs jobs;
    const double* xlag;   // [n_eta] Gauss-Laguerre nodes
    const double* wlag;   // [n_eta] w e^x
    const double* tleg;   // [n_tau]
    const double* wleg;   // [n_tau]
    const int* paths;     // [n_paths] global index of each local path
    const double* bvec;
    const double* vvec;
    double* nodes;        // [job][n_fields][n_nodes]
    int* jst;             // [job][2][n_nodes] first stencil node at rA, rB (-1 beyond r_max)
    int* n_act;           // [job] nodes in the active eta prefix
};

// k_2c_interp: the contraction operands of one position, once per job (f_a
// interpolated once per radial function and node, then scaled by the
// Legendre factor of every block s it enters):
//   AT[job][rowT_off[s] + i][p] = f_a(r_A(p)) Pbar_{l_a}^s(cos theta_A(p)),  a = radT_off[s] + i
//   BT[job][rowP_off[t] + i][p] = f_b(r_B(p)) Pbar_{l_b}^t(cos theta_B(p)),  b = radP_off[t] + i
// for active nodes p < n_act (node-contiguous rows, FP64, or FP32 in the mixed form).
struct InterpArgs {
    const Meta2C* m;
    const double* phiT_T;   // [nrT+1][nfT] target radial functions, transposed
    const double* phiT_P;   // [nrP+1][nfP]
    const int2* rinfoT;     // [rowsT] (radial index a, node field of Pbar_{l_a}^s)
    const int2* rinfoP;     // [rowsP]
    const double* nodes;
    const int* jst;
    const int* n_act;
    void* AT;               // [job][rowsT][n_nodes] double or float
    void* BT;               // [job][rowsP][n_nodes]
};

struct ContractArgs {
    const Meta2C* m;
    int n_jobs;
    const int2* tiles;      // [n_tiles] (s | t << 8, a0 | b0 << 16)
    const void* AT;         // interpolated operands (InterpArgs)
    const void* BT;
    const double* nodes;
    const int* n_act;
    double* tmol;           // [job][n_split][n_tmol]: partial sums over the node ranges
};

struct AssembleArgs {
    const Meta2C* m;
    Jobs jobs;
    const int* paths;
    const double* bvec;
    const double* vvec;
    const double* epsT;     // [NT]
    const double* epsP;     // [NP]
    const double* tmol;     // [job][n_split][n_tmol]: range 0 holds the sum (k_2c_reduce)
    double2* S;             // [path][slot][N*N] column-major
    double2* LU;            // copy of S for the factorisation
    double2* H;             // [path][slot][N*N] row-major
};

// S-norm-conserving form: dK = (K(z + dz) - K(z - dz)) / (2 dz) from two
// slots of S, then H <- (H + H^dag)/2 - (i v / 2) dS/dz in place
struct SymArgs {
    int N, NT, NP;
    int path0;              // first local path of the launch (grid y: paths)
    const int* paths;
    const double* vvec;
    double2* S;             // [path][slot][N*N] column-major
    double2* H;             // [path][slot][N*N] row-major
    double2* dK;            // [path][2][NT*NP] row-major
    int slot_p, slot_m;     // k_2c_dk: slots holding S at z + dz and z - dz
    int slot;               // k_2c_symm: slot whose H is replaced
    int which;              // dK buffer written / read
    double inv_2dz;
};

struct SetupBatchArgs {     // Frow, G, phases of one centre for the jobs of a launch
    const Meta* meta;
    Tables tb;
    Jobs jobs;
    const int* paths;
    int parity;             // -1: the other nucleus sits at -R (projectile centre)
    double* Frow;           // [job][n_frow]
    double* G;              // [job][n_g]
    double2* PH;            // [job][N_centre]
    int nbF, nbP;
};

struct DirectArgs {         // D_T and D_P blocks of H from the per-job Frow / G / phases
    const Meta* mT;
    const Meta* mP;
    const Meta2C* m;
    Jobs jobs;
    const double* FrowT;
    const double* GT;
    const double2* PHT;
    const double* FrowP;
    const double* GP;
    const double2* PHP;
    int n_frowT, n_gT, n_frowP, n_gP;
    double2* H;
};

// Blocked LU with partial pivoting of the S copies, one panel of kLUPanel
// columns per pass: k_lu_panel factors the panel (rows k0..N-1) in registers,
// k_lu_swap_trsm applies its row swaps to the other columns and solves the
// U12 block row, k_lu_update subtracts L21 U12 from the trailing matrix on
// MFMA.  perm accumulates the swaps as a row gather (y_perm[i] = y[perm[i]]).
constexpr int kLUPanel = 16;
constexpr int kLUMaxN = 2048;       // up to four rows per thread in the 512-thread panel kernel
// panel width of the factorisation of an N x N matrix: kLUPanel up to 1024
// rows (two rows per thread), half of it up to kLUMaxN (four rows per thread)
int lu_panel_width(int N);

// Overlap matrices S = [[I, K], [K^dagger, I]]: while every |K_ij| <= 1,
// partial pivoting keeps the diagonal 1 as the pivot of each of the first
// N_T columns (ties go to the lowest row), so those columns factor with
// L21 = K^dagger, U12 = K, L11 = U11 = I, and the rest is the LU of the
// Schur complement I - K^dagger K.  k_lu_check decides this per matrix
// (skip = 1) on the device; the Schur update then is one GEMM (k_lu_update
// with nb = N_T) and the panel steps of the first N_T columns return at once,
// while a matrix that fails the test takes those panel steps instead: the
// pivots are those of the general algorithm either way.
struct LUStepArgs {
    int N, k0, nb;          // panel columns k0 .. k0 + nb - 1 (k_lu_update: any nb)
    Jobs jobs;
    double2* LU;            // [path][slot][N*N] column-major, factorised in place
    int* piv;               // [path][slot][N] LAPACK-style pivot rows (0-based)
    int* perm;              // [path][slot][N]
    const int* paths;
    int* flag;              // [1] first singular path + 1, [2] its pivot column
    int* skip;              // [path][slot] 1: the first nt columns factor without pivoting (k_lu_check)
    int nt;                 // N_T (k_lu_check)
    int skip_mode;          // 0: run; 1: return where skip is set; 2: return where it is not
};

// M = S^{-1} H from the LU of S: the explicit form of Eq. INV, N right-hand sides
struct RhsArgs {
    int N;
    Jobs jobs;
    const double2* LU;      // [path][slot][N*N] column-major, P S = L U
    const int* perm;        // [path][slot][N] row i of P S is row perm[i] of S
    const double2* H;       // [path][slot][N*N] row-major
    double2* M;             // [path][slot][N*N] row-major
};

// One path's matrices for the stage kernels: slot s of the path starts at
// s * N * N (s * N for perm) from these bases.
struct PathMats {
    int N;
    int path;               // global path index (row of X, u, Y)
    const double2* H;       // H, or M = S^{-1} H when the stage does not solve
    const double2* LU;
    const int* perm;        // row order of the product (nullptr: identity)
};

// A stage for every path of pm[0 .. n_paths): the paths may differ in N (one
// launch over every basis-size group), N_max bounds them all.
struct Stage2CArgs {
    int N_max, n_pad, stage;
    double h;
    int slot;               // coupling slot used by this stage
    const PathMats* pm;
    const double* vvec;
    int solve;              // 1: y = U^{-1} L^{-1} P (H u); 0: y = M u
    // graph replays: h = hdev[3 * *step + 2] instead of h (nullptr: h)
    const double* hdev;
    const int* step;
    const double2* u_in;
    double2* Y;             // [n_traj][n_pad] P (H u) between the two kernels of a stage
    double2* X;
    double2* Xacc;
    double2* u_out;
    int* flag;
};

hipError_t launch_2c_nodes(const NodeArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_interp(const InterpArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_contract(const ContractArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
// adds the node-range partial sums of tmol into range 0 (nothing when n_split is 1)
hipError_t launch_2c_reduce(double* tmol, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_assemble(const AssembleArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_setup_batch(const SetupBatchArgs& a, const Meta& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_direct(const DirectArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_lu_panel(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_lu_swap_trsm(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_lu_update(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
// skip[matrix] = (max |L21| <= 1 over the first nt columns); where set, also
// perm = identity and piv[j] = j for j < nt
hipError_t launch_lu_check(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_lu_rhs(const RhsArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_hu(const Stage2CArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_solve(const Stage2CArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_finish(const double2* X, const double2* S, int N, int n_pad, const int* paths, int n_paths,
                            int slot, double* P, double* norm, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_transpose_copy(const double2* src_colmajor, double2* dst_rowmajor, int N, hipStream_t st);
hipError_t launch_2c_dk(const SymArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_2c_symm(const SymArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev = LaunchEv{});

}  // namespace wpccc

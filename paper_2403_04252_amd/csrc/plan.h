// Plan layout and kernel launchers of the one-centre path (internal).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <vector>

#include "wpccc_impl.h"

namespace wpccc {

constexpr int kMaxL = 10;            // largest l of a basis
constexpr int kMaxLam = 2 * kMaxL;   // largest multipole order
constexpr int kMaxPb = (kMaxLam + 1) * (kMaxLam + 2) / 2;
constexpr int kSlots = 3;            // couplings kept for the diagnostic entry point
constexpr int kStageThreads = 256;
// dynamic LDS a stage workgroup may request: the CU's 160 KB less room for
// the kernels' few static LDS words
constexpr int kMaxDynLds = 160 * 1024 - 1024;
constexpr int kRowsPerBlock = 8;     // output rows n' per workgroup of k_apply (and the untimed default of k_stage)
constexpr int kApplyRowsLarge = 4;   // k_apply's rows where kRowsPerBlock does not fit the LDS
// row tilings the stage kernels are built for (X-macro over the values)
#define WPCCC_STAGE_ROWS(X) X(4) X(5) X(6) X(7) X(8) X(10) X(12) X(16)
constexpr int kStageRowsList[] = {4, 5, 6, 7, 8, 10, 12, 16};
// row tilings of the large-basis form (angular factors from global memory)
#define WPCCC_STAGE_ROWS_GG(X) X(1) X(2) X(4)
constexpr int kStageRowsGG[] = {1, 2, 4};
constexpr int kNumStageRows = sizeof(kStageRowsList) / sizeof(kStageRowsList[0]);
constexpr int kChunkSteps = 64;                 // RK4 steps per prologue launch
constexpr int kChunkPoints = 2 * kChunkSteps + 1;  // z_0, z_mid_0, z_1, ..., z_n

// Per-basis sizes passed to kernels by value.
//
// Row layout ("Frow") of the radial integrals of one output l': the matrix
// F_l'[n'][e], n' < N_l', e < nV[l'], whose columns run over the blocks
// (l, lambda) in the order l = 0..l_max, lambda = |l-l'|..l+l' step 2, each
// block holding N_l columns (the radial index n of the input state):
//   F_l'[n'][e0(l, lambda) + n] = F_{(l' n'), (l n), lambda}(R)     (Eq. D2)
// The moment tables use the same layout per grid node k.
// Angular factors ("G") of one output l': the matrix G_l'[q'][g], q' = m'+l',
// g < gcols[l'], over the same blocks with 2l+1 columns (q = m+l) each:
//   G_l'[q'][g0(l, lambda) + q] = c(l'm', lm, lambda) Pbar_lambda^|m'-m|(cos Theta).
struct Meta {
    int l_max, lam_max, n_r, n_f, n_states, n_frow, n_g, n_chunks, n_cols, n_gcols;
    double r_max;
    int n_l[kMaxL + 1];
    int state_off[kMaxL + 1];
    int rad_off[kMaxL + 1];   // first radial index of each l
    int nV[kMaxL + 1];        // columns of F_l'
    int frow_off[kMaxL + 1];  // offset of F_l' in a Frow array / table row
    int col_off[kMaxL + 1];   // offset of l' in col_lam
    int gcols[kMaxL + 1];     // columns of G_l'
    int g_off[kMaxL + 1];     // offset of G_l' in a G array
    int gcol_off[kMaxL + 1];  // offset of l' in gcol_info
    int xs_off[kMaxL + 1];    // LDS position of x'_{l, q=0, n=0} in the stage kernels
    int xs_stride[kMaxL + 1]; // LDS stride between q rows of l: N_l rounded up to an odd number
    int n_xs;                 // LDS length (complex) of x' in the stage kernels
};

__host__ __device__ inline int pb_index(int lam, int mu) { return lam * (lam + 1) / 2 + mu; }

// G column info: x = e0 | (N_l << 16) (F column block start, block width),
// y = LDS position of x'_{l, q, 0} (the input states the column contracts
// with) in the stage kernels' padded layout (xs_off, xs_stride)
__host__ __device__ inline int2 gcol_pack(int e0, int nl, int xoff) { return make_int2(e0 | (nl << 16), xoff); }

// Basis tables shared by every launch of a plan.
struct Tables {
    const double2* tab;     // [n_r+1][n_frow]: (A_k, B_(k+1)) per Frow entry (FP64 plans)
    const float2* tab32;    // [n_r+1][n_frow]: the scaled FP32 form (reduced-precision plans, else NULL):
                            //   (A_k / r_k^(lam+1), B_(k+1) r_(k+1)^lam)
    const double* ftab;     // [n_r+1][n_frow]: F(r_k) on the grid nodes (interpolated-F plans, else NULL)
    const int* col_lam;     // [n_cols] lambda of each Frow column, per l'
    const int2* gcol_info;  // [n_gcols] gcol_pack of each G column, per l'
    const double* gcoef;    // [n_g] c(l'm', lm, lambda), (-1)^mu folded in for mu < 0
    const int* gpb;         // [n_g] pb_index(lambda, |mu|) or -1
    const double* eps;      // [N] state energies
    const int* st_rad;      // [N] radial index of each state
    const int* st_xs;       // [N] LDS position of each state's x' (xs_off, xs_stride)
    const double* rad_eps;  // [n_f] energy of each radial function
    const double* bvec;     // [n_traj]
    const double* vvec;     // [n_traj]
};

// Per (path, z-point) quantities shared by every workgroup of a stage,
// computed once by k_prologue for all points of a propagation chunk:
//   kidx[j][p]                grid node of R (last r_k <= R)
//   rpow[j][p][2 lam]         R^-(lam+1) at 2 lam, R^lam at 2 lam + 1 (FP64 table);
//                             (r_k/R)^(lam+1) and (R/r_(k+1))^lam (scaled FP32 table);
//                             interpolated F: the five Lagrange weights of the
//                             stencil starting at node kidx (R < r_max), or
//                             kidx = -1 and (r_max/R)^(lam+1) at lam (R >= r_max)
//   pbar[j][p][n_pb]          Pbar_lam^mu(cos Theta)
//   ph[j][p][n_f]             exp(i eps_f z / v) per radial function
struct PointArrays {
    int* kidx;
    double* rpow;
    double* pbar;
    double2* ph;
    int n_pts;      // capacity in points per path
};

constexpr int kRpow = 2 * (kMaxLam + 1);

// One row tile of a one-centre stage grid (rows [row0, row0 + nrows) of the
// l' block) with the per-l' offsets the stage kernels need, so that a
// workgroup gets its work from one 64-byte load.  The tiles of one path are
// listed in l' order; vo = sum of N_l^2 over l < l' (model potential blocks).
struct alignas(64) StageTile {
    int lp, row0, nrows, nmp;
    int nV, gcols, frow_off, col_off;
    int g_off, gcol_off, state_off, rad_off;
    int n_l, xs_off, xs_stride, vo;
};

struct StageArgs {
    const Meta* meta;     // device copy (indexed per lane: kept out of kernel arguments)
    const StageTile* tiles;  // [nwg] the row tiles of one path for this launch's tiling
    int nwg;
    Tables tb;
    PointArrays pt;
    double Zp;
    int p;                // z-point of this stage's couplings in pt
    double h;
    int n_pad;
    int stage;            // 1..4
    int gg;               // large-basis form: angular factors read from global memory (k_stage only)
    int traj0;
    int n_paths;          // paths of a k_stage launch (set by launch_stage)
    const double2* u_in;  // stage input   [n_traj][n_pad]
    double2* X;           // amplitudes    [n_traj][n_pad]
    double2* Xout;        // stage 4 writes the step's result here (NULL: in place in X)
    double2* Xacc;        // accumulator   [n_traj][n_pad]
    double2* u_out;       // next input    [n_traj][n_pad]
    int* flag;            // non-finite latch
    // graph replays: h = hdev[*chunk * kChunkSteps + hidx] instead of h
    const double* hdev;
    const int* chunk;
    int hidx;
    // radial-integral cache of the stage kernels (kFcSlots): fc_cur holds F
    // at this stage's point for every path ([n_traj][n_frow], double, or
    // float with the scaled FP32 table; NULL: the stage forms F from the
    // moment table itself); fc_next (may be NULL) receives F at point p_next,
    // formed from the moment table after the stage's own work
    const void* fc_cur;
    void* fc_next;
    int p_next;
    // operator application (k_apply): y = O v with O = M(z_p) (deriv 0),
    // (b/R) dM/dR (deriv 1) or (-z b/R^3) dM/dcos(Theta) (deriv 2) applied to
    // v = cu1 u_in + cu2 u_in2 (u_in2 may be NULL), then
    //   out = alpha y + w[0] + ... + w[3]   (out may be NULL, unused w[k] NULL)
    //   grad[(j * kGradSlots + gslot) * gridDim.x + blockIdx.x] += this
    //   workgroup's share of 2 gamma Re(d^H y), d = cd1 dv + cd2 dv2
    //   (grad may be NULL; gslot 0 or 1)
    // and, with model != 0, the shares of 2 gamma Re(d^H dM/da v) and
    // 2 gamma Re(d^H dM/dc v) in slots 2 and 3, from the radial blocks of the
    // model potential (one-centre plans):
    //   va[vo(l) + n' N_l + n] = -sum_i w_i r_i f f e^{-c r_i}       (d DeltaV / da)
    //   vc[vo(l) + n' N_l + n] = +a sum_i w_i r_i^2 f f e^{-c r_i}   (d DeltaV / dc)
    // with vo(l) = sum_{l'' < l} N_l''^2
    int deriv;
    double z;             // z of the point (deriv 1, 2)
    double cu1, cu2;
    const double2* u_in2;
    double alpha, gamma;
    const double2* w[4];
    double2* out;
    const double2* dv;
    const double2* dv2;
    double cd1, cd2;
    double* grad;         // [n_traj][kGradSlots][grid x] shares
    int gslot;
    int model;
    const double* va;
    const double* vc;
};

// Radial-integral cache of a one-centre propagation: F_l'(R) of Eq. D2 in the
// row layout for every path at two points, slot 0 holding the step's end
// points and slot 1 its midpoints.  Of the four stages of a step (points z,
// z_mid, z_mid, z_new), stage 1 reads slot 0 and fills slot 1 with F(z_mid),
// stage 2 reads slot 1, stage 3 reads slot 1 and fills slot 0 with F(z_new),
// stage 4 reads slot 0; k_fpoint fills slot 0 at the first point of a run of
// steps.  So the moment table is read at the two new points of each step,
// while the stage that consumes a point's couplings has them ready.
constexpr int kFcSlots = 2;

// gradient share slots of k_apply per path: b (deriv 1), b (deriv 2), a, c
constexpr int kGradSlots = 4;

// ints between the barrier counters of two paths: one 256-byte line each, so
// that the polls of different paths do not contend for one memory line
constexpr int kBarStride = 64;

// Up to three operator applications of one k_apply launch (grid z selects
// one; they share the launch's point slot and run side by side).
struct ApplyArgs {
    StageArgs s[3];
};

// Persistent form of a propagation chunk (k_chunk): every workgroup of the
// stage grid stays resident for all steps of the chunk and the workgroups of
// one path meet at a barrier (bar[path], counted with agent-scope atomics)
// between stages, instead of ending the kernel.
struct ChunkArgs {
    StageArgs s;          // per-plan fields; p, h, stage, u_in, u_out are set per stage
    double2* Ua;
    double2* Ub;
    int n_steps;
    double h[kChunkSteps];
    int* bar;             // [n_traj][kBarStride], zero at launch (counter of path j at bar[j * kBarStride])
    int n_traj;
};

struct SetupArgs {
    const Meta* meta;
    Tables tb;
    double z;
    int j;                // path
    double* Frow;         // [n_frow]
    double* G;            // [n_g]
    double2* PH;          // [N]
    int nbF, nbP;         // block ranges: Frow entries, phases, then G
};

struct PrologueArgs {
    const Meta* meta;
    Tables tb;
    PointArrays pt;
    double z[kChunkPoints];  // z of each point of the chunk
    int n;                   // points in this launch
    int traj0;
    // graph replays: z = zdev[*chunk * kChunkPoints + p] instead of z[p]
    const double* zdev;
    const int* chunk;
};

// Device tables of one centre's basis (moment tables, column maps, angular
// coefficients, energies), built once per basis by centre_build().
struct Centre {
    Meta meta{};
    Meta* d_meta = nullptr;
    double *d_eps = nullptr, *d_gcoef = nullptr, *d_rad_eps = nullptr;
    int *d_col_lam = nullptr, *d_gpb = nullptr, *d_st_rad = nullptr, *d_st_xs = nullptr;
    int2* d_gcol = nullptr;
    double2* d_tab = nullptr;     // FP64 moment table (NULL once a scaled FP32 table replaces it)
    float2* d_tab32 = nullptr;    // scaled FP32 moment table (reduced-precision one-centre plans)
    double* d_ftab = nullptr;     // F on the grid nodes (interpolated-F one-centre plans)
    long long bytes = 0;
    Tables tables(const double* bvec, const double* vvec) const {
        Tables t;
        t.tab = d_tab;
        t.tab32 = d_tab32;
        t.ftab = d_ftab;
        t.col_lam = d_col_lam;
        t.gcol_info = d_gcol;
        t.gcoef = d_gcoef;
        t.gpb = d_gpb;
        t.eps = d_eps;
        t.st_rad = d_st_rad;
        t.st_xs = d_st_xs;
        t.rad_eps = d_rad_eps;
        t.bvec = bvec;
        t.vvec = vvec;
        return t;
    }
};

// Events of one timed launch: recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so their interval is the kernel's execution.
struct LaunchEv {
    hipEvent_t a = nullptr, b = nullptr;
};
#define WPCCC_LAUNCH(ev, kernel, grid, block, smem, st, ...)                                        \
    do {                                                                                          \
        if ((ev).a)                                                                               \
            hipExtLaunchKernelGGL(kernel, grid, block, smem, st, (ev).a, (ev).b, 0, __VA_ARGS__); \
        else                                                                                      \
            hipLaunchKernelGGL(kernel, grid, block, smem, st, __VA_ARGS__);                       \
    } while (0)

// Optional per-kernel timing with HIP events recorded on the launch stream
// (wpccc_plan_timing / wpccc_plan_kernel_time).
enum KernelId {
    kStage = 0, kSetup, kDense, kProb, kMoments, kPrologue,
    k2cNodes, k2cInterp, k2cContract, k2cAssemble, k2cSetup, k2cDirect, kLuPanel, kLuSwap, kLuUpdate, k2cHu, k2cSolve, k2cFinish,
    kChunk, k2cReduce, kFpoint, kChannels, kLuCheck, kLuRhs, k2cDk, k2cSymm, kNumKernels
};
extern const char* const kKernelNames[kNumKernels];

struct KernelTimer {
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    bool on = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    // events for one launch of `kernel` (none when timing is off)
    LaunchEv open(int kernel);
    void recycle_all();
    // total time and count of the finished launches of `kernel`, which are then forgotten
    int take(int kernel, double* total_ms, long long* launches);
    ~KernelTimer();
};

// Reaction channels of the states (observables.hip): elastic, target
// excitation, target continuum, capture, projectile continuum, total.
constexpr int kNumChannels = 6;
constexpr unsigned char kChElastic = 0, kChExcitation = 1, kChTargetCont = 2, kChCapture = 3, kChProjCont = 4,
                        kChPadding = 255;

// Per-plan tables of the observables: a channel code per state of every path
// ([n_traj][n_pad], kChPadding beyond N_j), the group of every path (paths
// sharing the basis pair and the speed) and each group's paths by increasing b.
struct Observables {
    int n_traj = 0, n_pad = 0, n_groups = 0;
    std::vector<int> group_of;
    unsigned char* d_code = nullptr;
    int* d_order = nullptr;
    int* d_gstart = nullptr;
    double* d_b = nullptr;
    long long bytes = 0;
};
int obs_build(Observables& o, int n_traj, int n_pad, const std::vector<unsigned char>& codes,
              const std::vector<int>& group_of, const std::vector<double>& b);
void obs_free(Observables& o);
// chan [n_traj][kNumChannels] from P [n_traj][n_pad]; sigma [n_groups][kNumChannels] (may be NULL)
hipError_t launch_observables(const Observables& o, const double* P, double* chan, double* sigma, hipStream_t st,
                              const LaunchEv& ev = LaunchEv{});

// centre.hip
// model_a != 0 adds DeltaV = -a e^{-c r}/r (block diagonal in l, m) to the
// lambda = 0 moments of the equal-l blocks, so that every use of the tables
// sees D_T + DeltaV (projectile charge Zp)
// Radial-integral forms a centre's tables can take (centre_build):
enum RadialForm {
    kRadialMoments = 0,   // FP64 moment table: Eq. D2's quadrature at the exact R
    kRadialMoments32 = 1, // its scaled FP32 form (Tables::tab32)
    kRadialInterp = 2,    // F on the grid nodes, five-point interpolation at R (Tables::ftab)
};
int centre_build(const HostBasis& hb, hipStream_t st, Centre& c, double model_a = 0.0, double model_c = 0.0,
                 double Zp = 1.0, int form = kRadialMoments);
// radial blocks va, vc of the model potential (layout of StageArgs::va, vc)
void model_blocks(const HostBasis& hb, double a, double c, std::vector<double>& va, std::vector<double>& vc);
void centre_free(Centre& c);

// device allocation with error text; adds to `total`
int dev_alloc_bytes(void** p, size_t bytes, long long& total);
template <typename T>
inline int dev_alloc(T** p, size_t count, long long& total) {
    return dev_alloc_bytes(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T), total);
}
int launched(hipError_t e, const char* what);

// sustained FP64 / FP32 16x16x4 MFMA rates of the current device in TFLOP/s,
// synchronising st (kernels_2c.hip)
hipError_t measure_mfma(double* tflops_f64, double* tflops_f32, hipStream_t st);

// two-centre plan (plan2c.hip)
struct Plan2C;
int plan2c_create(const wpccc_basis_t* targets, const wpccc_basis_t* projectiles, int n_sets, int n_traj,
                  const int* set_of_traj, const double* b, const double* v, const wpccc_plan_opts& o,
                  KernelTimer* timer, hipStream_t st, Plan2C** out);
void plan2c_destroy(Plan2C* p);
int plan2c_info(Plan2C* p, int* n_traj, int* n_states, int* n_pad, long long* bytes);
int plan2c_path_info(Plan2C* p, int j, int* n_states, int* n_target);
int plan2c_status(Plan2C* p, hipStream_t st);
// A X = B for batch column-major A with n row-major right-hand sides (plan2c.hip)
int lu_solve_batched(int n, int batch, const void* A, const void* B, void* X, hipStream_t st);
int plan2c_couplings(Plan2C* p, int j, double z, void* H, void* S, hipStream_t st);
int plan2c_step(Plan2C* p, void* X, double z, double h, hipStream_t st);
int plan2c_propagate(Plan2C* p, const double* zgrid, int n_points, void* X, void* P, void* norm, hipStream_t st);

// launchers (kernels_1c.hip)
hipError_t launch_prologue(const PrologueArgs& a, int n_traj_launch, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_moments(const double* r, const double* w, const double* phiT, const int* da,
                          const int* db, const int* dl, int n_r, int n_f, int n_frow, double2* tab,
                          hipStream_t st);
hipError_t launch_slot_setup(const SetupArgs& a, const Meta& host_meta, hipStream_t st, const LaunchEv& ev = LaunchEv{});
// rows: output rows n' per workgroup (4, 8 or 16; chosen per plan by timing)
hipError_t launch_stage(const StageArgs& a, const Meta& host_meta, int n_traj_launch, int smem, hipStream_t st,
                        const LaunchEv& ev = LaunchEv{}, int rows = kRowsPerBlock);
// F of Eq. D2 at point slot p of the prologue arrays for paths [traj0, traj0 +
// n_paths) into fc[j][n_frow] (the radial-integral cache; float elements with
// the scaled FP32 table, else double)
hipError_t launch_fpoint(const Meta* m, const Meta& host_meta, const Tables& tb, const PointArrays& pt, int p,
                         int traj0, int n_paths, void* fc, hipStream_t st, const LaunchEv& ev = LaunchEv{});
hipError_t launch_couplings_dense(const Meta* m, const Meta& host_meta, const double* Frow, const double* G,
                                  const double2* PH, double Zp, double2* H, hipStream_t st,
                                  const LaunchEv& ev = LaunchEv{});
hipError_t launch_probabilities(const double2* X, int n_traj, int n_states, int n_pad, double* P,
                                double* norm, hipStream_t st, const LaunchEv& ev = LaunchEv{});
// rows: kRowsPerBlock or kApplyRowsLarge; gg: the large-basis form with rows
// 4, 2 or 1 (a.tiles must be that tiling)
hipError_t launch_apply(const ApplyArgs& a, int n_ops, const Meta& host_meta, int n_traj_launch, int smem, int rows,
                        bool gg, hipStream_t st, const LaunchEv& ev = LaunchEv{});
// grad[j][0..2] = (a, c, b) sums of the k_apply shares gpart[j][kGradSlots][n_part]
// in a fixed order; one workgroup per path
hipError_t launch_grad_sum(const double* gpart, int n_part, double* grad, int n_traj, hipStream_t st);
// *chunk = value (reset) or *chunk += 1 (advance), one thread
hipError_t launch_chunk_counter(int* chunk, int reset, hipStream_t st);
hipError_t launch_table_shift(double2* tab, int n_frow, int n_r, const int* idx, const double* val, int count,
                              hipStream_t st);
// F on the grid nodes from a moment table (Tables::ftab)
hipError_t launch_table_nodes(const double2* tab, const int* dl, int n_frow, int n_r, double r_max, double* out,
                              hipStream_t st);
// scaled FP32 copy of a moment table (Tables::tab32); dl: multipole order of each entry
hipError_t launch_table_f32(const double2* tab, const int* dl, int n_frow, int n_r, double r_max, float2* out,
                            hipStream_t st);
hipError_t stage_set_smem_limit(int l_max, int bytes);
// k_chunk with `rows` rows per workgroup as one cooperative launch; returns
// hipErrorCooperativeLaunchTooLarge (and launches nothing) when the grid
// cannot be resident at once
hipError_t launch_chunk(const ChunkArgs& a, const Meta& host_meta, int smem, int rows, hipStream_t st,
                        const LaunchEv& ev = LaunchEv{});
// workgroups k_chunk needs for n_traj paths (rows per workgroup), and whether they fit at once
int chunk_grid(const Meta& host_meta, int n_traj, int rows);
bool chunk_fits(const Meta& host_meta, int n_traj, int rows, int smem);
// gg: the large-basis form (no angular factors in LDS)
int stage_smem_bytes(const Meta& m, int rows = kRowsPerBlock, bool gg = false);
// the row tiles of one path for `rows` rows per workgroup, l' order
void stage_tiles(const Meta& m, int rows, std::vector<StageTile>& out);
// k_stage's tiles: every l' block split into tiles of even size, of at most
// `rows` rows, or rows - 1 for the largest l' (from l_max down) while
// n_launch paths of such tiles still fit wg_slots resident workgroups (the
// larger l' blocks take longer per row, and a launch ends with its slowest
// workgroup)
void stage_tiles_balanced(const Meta& m, int rows, int n_launch, long long wg_slots, std::vector<StageTile>& out);
// resident k_stage workgroups per CU at `rows` rows and smem bytes of dynamic LDS (0: unknown)
int stage_wgs_per_cu(int rows, int smem);
// whether the stage kernels can use `rows` rows per workgroup for this basis
// (every output of a workgroup needs a lane of the phase-3 reduction)
bool stage_rows_fit(const Meta& m, int rows);
// LDS of k_chunk: the stage layout plus the multipole order of each F column
int chunk_smem_bytes(const Meta& m, int rows);
int stage_chunks(const Meta& m, int rows);

}  // namespace wpccc

// C ABI: basis handles, the one-centre plan and the entry points; the
// two-centre plan lives in plan2c.hip and is reached through the same calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "plan.h"

namespace wpccc {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

}  // namespace wpccc

using namespace wpccc;

struct wpccc_plan_s {
    Plan2C* p2c = nullptr;   // set for a two-centre plan (everything below unused)
    Centre c;                // one-centre basis tables
    int n_traj = 0, n_pad = 0, batched = 1;
    double Zp = 1.0;
    std::vector<double> b, v;
    double *d_b = nullptr, *d_v = nullptr;
    int* d_flag = nullptr;
    double *d_Frow1 = nullptr, *d_G1 = nullptr;  // diagnostic couplings scratch
    double2* d_PH1 = nullptr;
    double2 *d_Ua = nullptr, *d_Ub = nullptr, *d_Xacc = nullptr;
    int* d_kidx = nullptr;
    double *d_rpow = nullptr, *d_pbar = nullptr;
    double2* d_ph = nullptr;
    void* d_fc = nullptr;    // [kFcSlots][n_traj][n_frow] radial-integral cache of the stage kernels
                             // (double; float for the scaled FP32 table)
    // model potential blocks and adjoint workspace (allocated on first use)
    double *d_va = nullptr, *d_vc = nullptr;
    int ckpt_every = 0;
    int adj_K = 0, adj_nck = 0;
    double2 *d_lam = nullptr, *d_nu = nullptr;   // [2][n_traj][n_pad], [3][n_traj][n_pad]
    double2 *d_ckpt = nullptr, *d_seg = nullptr;  // checkpoints; segment store (states, stage inputs)
    // graph replay of 64-step chunks (wpccc_propagate)
    bool use_graph = false, capturing = false;
    hipStream_t gstream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const double2* gX = nullptr;
    int g_cap = 0;                      // chunks the z/h arrays hold
    double *d_zall = nullptr, *d_hall = nullptr, *h_zh = nullptr;  // h_zh: pinned staging
    int* d_chunk = nullptr;
    hipEvent_t g_copied = nullptr;
    long long bytes = 0;
    int stage_smem = 0;       // k_apply (apply_rows rows)
    int apply_rows = kRowsPerBlock;
    bool apply_ok = true;     // k_apply's LDS fits (wpccc_adjoint is available)
    int stage_rows = kRowsPerBlock;
    int stage_smem_rows = 0;  // k_stage with stage_rows
    // propagation chunks kernel by kernel (WPCCC_LAUNCH_STAGES) or as one
    // persistent k_chunk launch (WPCCC_LAUNCH_PERSISTENT)
    int launch = WPCCC_LAUNCH_STAGES;
    bool mixed = false;       // scaled FP32 moment table (WPCCC_MIXED): per-stage launches only, no adjoint
    bool interp = false;      // F on the grid nodes, five-point interpolation (WPCCC_RADIAL_INTERP)
    int chunk_smem = 0;       // k_chunk with stage_rows
    int* d_bar = nullptr;     // [n_traj][kBarStride] path barrier counters of k_chunk
    double* d_gpart = nullptr;  // [n_traj][kGradSlots][n_chunks] per-workgroup gradient shares (k_apply)
    StageTile* d_tiles = nullptr;  // the row tiles of every tiling in kStageRowsList, one after another
    Observables obs;               // channel codes and path groups (wpccc_observables)
    int tile_off[kNumStageRows] = {}, tile_n[kNumStageRows] = {};
    // k_stage's balanced tilings (stage_tiles_balanced); k_apply keeps the plain ones
    int tile_off_bal[kNumStageRows] = {}, tile_n_bal[kNumStageRows] = {};
    // large-basis form (no regular tiling fits the LDS): angular factors read
    // from global memory, tilings of kStageRowsGG rows after the regular ones
    bool gg = false;
    int tile_off_gg[3] = {}, tile_n_gg[3] = {};
    // stage kernels take F from the radial-integral cache (else every stage
    // forms F from the moment table); required by the FP32-table,
    // interpolated-F and large-basis forms, timed against the direct form
    // otherwise
    bool fcache = true;
    int cache_req = WPCCC_CACHE_AUTO;
    KernelTimer timer;

    Tables tables() const { return c.tables(d_b, d_v); }
    PointArrays points() const {
        PointArrays q;
        q.kidx = d_kidx;
        q.rpow = d_rpow;
        q.pbar = d_pbar;
        q.ph = d_ph;
        q.n_pts = kChunkPoints;
        return q;
    }
};

namespace {

void free_plan(wpccc_plan_s* p) {
    if (!p) return;
    if (p->p2c) plan2c_destroy(p->p2c);
    obs_free(p->obs);
    centre_free(p->c);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->gstream) (void)hipStreamDestroy(p->gstream);
    if (p->g_copied) (void)hipEventDestroy(p->g_copied);
    if (p->h_zh) (void)hipHostFree(p->h_zh);
    if (p->d_zall) (void)hipFree(p->d_zall);
    if (p->d_hall) (void)hipFree(p->d_hall);
    if (p->d_chunk) (void)hipFree(p->d_chunk);
    void* bufs[] = {p->d_b,    p->d_v,    p->d_flag, p->d_Frow1, p->d_G1,   p->d_PH1,  p->d_Ua,
                    p->d_Ub,   p->d_Xacc, p->d_kidx, p->d_rpow,  p->d_pbar, p->d_ph,   p->d_va,
                    p->d_vc,   p->d_lam,  p->d_nu,   p->d_ckpt,  p->d_seg,  p->d_bar,  p->d_gpart,
                    p->d_tiles, p->d_fc};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    delete p;
}

// Per-point quantities for z[0..n) of paths [j0, j0+nj) into point slots 0..n-1.
int enqueue_prologue(wpccc_plan_s* p, const double* z, int n, int j0, int nj, hipStream_t st) {
    PrologueArgs a;
    a.meta = p->c.d_meta;
    a.tb = p->tables();
    a.pt = p->points();
    for (int i = 0; i < n; ++i) a.z[i] = z[i];
    a.n = n;
    a.traj0 = j0;
    a.zdev = p->capturing ? p->d_zall : nullptr;
    a.chunk = p->capturing ? p->d_chunk : nullptr;
    hipError_t e = launch_prologue(a, nj, st, p->timer.open(kPrologue));
    return launched(e, "k_prologue");
}

// The row tiles of a tiling (`rows` from kStageRowsList, or from
// kStageRowsGG in the large-basis form).
void set_tiles(const wpccc_plan_s* p, int rows, StageArgs& a) {
    if (p->gg) {
        for (int i = 0; i < 3; ++i)
            if (kStageRowsGG[i] == rows) {
                a.tiles = p->d_tiles + p->tile_off_gg[i];
                a.nwg = p->tile_n_gg[i];
            }
        return;
    }
    for (int i = 0; i < kNumStageRows; ++i)
        if (kStageRowsList[i] == rows) {
            a.tiles = p->d_tiles + p->tile_off[i];
            a.nwg = p->tile_n[i];
        }
}

// Fields of a stage launch shared by every stage of a propagation.
StageArgs stage_args(const wpccc_plan_s* p, int j0, double2* X) {
    StageArgs a{};
    a.meta = p->c.d_meta;
    set_tiles(p, p->stage_rows, a);
    if (!p->gg)
        for (int i = 0; i < kNumStageRows; ++i)
            if (kStageRowsList[i] == p->stage_rows) {
                a.tiles = p->d_tiles + p->tile_off_bal[i];
                a.nwg = p->tile_n_bal[i];
            }
    a.gg = p->gg ? 1 : 0;
    a.tb = p->tables();
    a.pt = p->points();
    a.Zp = p->Zp;
    a.n_pad = p->n_pad;
    a.traj0 = j0;
    a.X = X;
    a.Xacc = p->d_Xacc;
    a.flag = p->d_flag;
    return a;
}

// Slot s of the radial-integral cache (FCache in plan.h).
void* fc_slot(const wpccc_plan_s* p, int s) {
    const size_t elem = p->mixed ? sizeof(float) : sizeof(double);
    return static_cast<char*>(p->d_fc) + (size_t)s * p->n_traj * p->c.meta.n_frow * elem;
}

// F at point slot `point` into cache slot `slot` (0: the start of a run of
// cached steps) for paths [j0, j0+nj).
int enqueue_fpoint(wpccc_plan_s* p, int j0, int nj, int point, hipStream_t st, int slot = 0) {
    hipError_t e = launch_fpoint(p->c.d_meta, p->c.meta, p->tables(), p->points(), point, j0, nj, fc_slot(p, slot), st,
                                 p->timer.open(kFpoint));
    return launched(e, "k_fpoint");
}

// fc_cur / fc_next: cache slots (-1: none; fc_cur -1 forms F from the table)
int enqueue_stage(wpccc_plan_s* p, int j0, int nj, int stage, int point, int step, double h, const double2* u_in,
                  double2* X, double2* u_out, hipStream_t st, double2* Xout = nullptr, int fc_cur = -1,
                  int fc_next = -1, int p_next = 0) {
    StageArgs a = stage_args(p, j0, X);
    a.fc_cur = fc_cur >= 0 ? fc_slot(p, fc_cur) : nullptr;
    a.fc_next = fc_next >= 0 ? fc_slot(p, fc_next) : nullptr;
    a.p_next = p_next;
    a.Xout = Xout;
    a.p = point;
    a.h = h;
    a.stage = stage;
    a.u_in = u_in;
    a.u_out = u_out;
    a.hdev = p->capturing ? p->d_hall : nullptr;
    a.chunk = p->capturing ? p->d_chunk : nullptr;
    a.hidx = step;
    hipError_t e = launch_stage(a, p->c.meta, nj, p->stage_smem_rows, st, p->timer.open(kStage), p->stage_rows);
    return launched(e, "k_stage");
}

// Steps 0..ns-1 of the current prologue chunk (step lengths h[i]) for paths
// [j0, j0+nj) as one persistent k_chunk launch with `rows` rows per workgroup.
int enqueue_chunk(wpccc_plan_s* p, double2* X, int j0, int nj, const double* h, int ns, int rows, int smem,
                  hipStream_t st) {
    ChunkArgs c{};
    c.s = stage_args(p, j0, X);
    c.Ua = p->d_Ua;
    c.Ub = p->d_Ub;
    c.n_steps = ns;
    for (int i = 0; i < ns; ++i) c.h[i] = h[i];
    c.bar = p->d_bar;
    c.n_traj = nj;
    WPCCC_HIP_CHECK(hipMemsetAsync(p->d_bar, 0, (size_t)nj * kBarStride * sizeof(int), st));
    return launched(launch_chunk(c, p->c.meta, smem, rows, st, p->timer.open(kChunk)), "k_chunk");
}

// One RK4 step of length h for paths [j0, j0+nj) with M at the points pz (z),
// pz+1 (z_mid) and pz+2 (z_new).  Stage inputs alternate between two buffers
// so that no stage reads what it writes.  cached: the stages take F from the
// radial-integral cache, whose slot 0 must hold F(pz) (enqueue_fpoint, or the
// previous cached step), and leave F(pz+2) in slot 0; otherwise every stage
// forms F from the moment table.
int enqueue_step(wpccc_plan_s* p, double2* X, int j0, int nj, int pz, double h, hipStream_t st, bool cached = true) {
    int rc;
    cached = cached && p->fcache;
    // the step's index within its chunk (graph replays read h at this index)
    const int step = pz / 2;
    const int c0 = cached ? 0 : -1, c1 = cached ? 1 : -1;
    if (p->interp) {
        // interpolated F: the cache is filled by k_fpoint at each new point
        if ((rc = enqueue_stage(p, j0, nj, 1, pz, step, h, X, X, p->d_Ua, st, nullptr, 0))) return rc;
        if ((rc = enqueue_fpoint(p, j0, nj, pz + 1, st, 1))) return rc;
        if ((rc = enqueue_stage(p, j0, nj, 2, pz + 1, step, h, p->d_Ua, X, p->d_Ub, st, nullptr, 1))) return rc;
        if ((rc = enqueue_stage(p, j0, nj, 3, pz + 1, step, h, p->d_Ub, X, p->d_Ua, st, nullptr, 1))) return rc;
        if ((rc = enqueue_fpoint(p, j0, nj, pz + 2, st, 0))) return rc;
        return enqueue_stage(p, j0, nj, 4, pz + 2, step, h, p->d_Ua, X, nullptr, st, nullptr, 0);
    }
    if ((rc = enqueue_stage(p, j0, nj, 1, pz, step, h, X, X, p->d_Ua, st, nullptr, c0, c1, pz + 1))) return rc;
    if ((rc = enqueue_stage(p, j0, nj, 2, pz + 1, step, h, p->d_Ua, X, p->d_Ub, st, nullptr, c1))) return rc;
    if ((rc = enqueue_stage(p, j0, nj, 3, pz + 1, step, h, p->d_Ub, X, p->d_Ua, st, nullptr, c1, c0, pz + 2)))
        return rc;
    if ((rc = enqueue_stage(p, j0, nj, 4, pz + 2, step, h, p->d_Ua, X, nullptr, st, nullptr, c0))) return rc;
    return WPCCC_OK;
}

bool path_hits_origin(const wpccc_plan_s* p, double z) {
    for (double b : p->b)
        if (!(std::sqrt(b * b + z * z) > 0.0)) return true;
    return false;
}

int check_grid(const double* zgrid, int n_points) {
    if (!zgrid || n_points < 2) {
        set_error("wpccc_propagate: need a z-grid of at least 2 points");
        return WPCCC_EINVAL;
    }
    for (int i = 0; i < n_points; ++i)
        if (!std::isfinite(zgrid[i]) || (i > 0 && !(zgrid[i] > zgrid[i - 1]))) {
            set_error("wpccc_propagate: z-grid must be finite and strictly increasing");
            return WPCCC_EINVAL;
        }
    return WPCCC_OK;
}

// Point slots of the adjoint's steps: steps [c0, c0 + kChunkSteps) share one
// prologue launch (point 2i is zgrid[c0+i], point 2i+1 the midpoint of step
// c0+i, as in wpccc_propagate); returns the first slot of step n, after a
// prologue launch when step n is not in the loaded chunk.
struct AdjointPoints {
    const double* zg;
    int n_steps;
    int loaded = -1;
    int slot(wpccc_plan_s* p, int n, hipStream_t st, int* rc) {
        const int c = n / kChunkSteps, c0 = c * kChunkSteps;
        if (c != loaded) {
            const int ns = std::min(kChunkSteps, n_steps - c0);
            double pts[kChunkPoints];
            for (int i = 0; i <= ns; ++i) {
                pts[2 * i] = zg[c0 + i];
                if (i < ns) pts[2 * i + 1] = 0.5 * (zg[c0 + i] + zg[c0 + i + 1]);
            }
            if ((*rc = enqueue_prologue(p, pts, 2 * ns + 1, 0, p->n_traj, st))) return 0;
            loaded = c;
        }
        return 2 * (n - c0);
    }
};

// One RK4 step of every path from x (point slots pz, pz+1, pz+2) that keeps
// its stage inputs u2, u3, u4 and writes its result to xn (x is only read).
int stored_step(wpccc_plan_s* p, int pz, double h, double2* x, double2* xn, double2* u2, double2* u3, double2* u4,
                hipStream_t st) {
    int rc;
    const int nj = p->n_traj;
    // the large-basis stage form takes F from the radial-integral cache:
    // F(pz) into slot 0 first, then the cached pattern of enqueue_step
    const bool c = p->gg;
    if (c && (rc = enqueue_fpoint(p, 0, nj, pz, st, 0))) return rc;
    const int c0 = c ? 0 : -1, c1 = c ? 1 : -1;
    if ((rc = enqueue_stage(p, 0, nj, 1, pz, 0, h, x, x, u2, st, nullptr, c0, c1, pz + 1))) return rc;
    if ((rc = enqueue_stage(p, 0, nj, 2, pz + 1, 0, h, u2, x, u3, st, nullptr, c1))) return rc;
    if ((rc = enqueue_stage(p, 0, nj, 3, pz + 1, 0, h, u3, x, u4, st, nullptr, c1, c0, pz + 2))) return rc;
    return enqueue_stage(p, 0, nj, 4, pz + 2, 0, h, u4, x, nullptr, st, xn, c0);
}

// Fields of a k_apply operation at point slot pt (z of the point).
StageArgs apply_args(const wpccc_plan_s* p, int pt, double z, int deriv) {
    StageArgs a{};
    a.meta = p->c.d_meta;
    set_tiles(p, p->apply_rows, a);
    a.tb = p->tables();
    a.pt = p->points();
    a.Zp = p->Zp;
    a.p = pt;
    a.n_pad = p->n_pad;
    a.traj0 = 0;
    a.flag = p->d_flag;
    a.deriv = deriv;
    a.z = z;
    a.cu1 = 1.0;
    a.cd1 = 1.0;
    a.gamma = 1.0;
    return a;
}

// One reverse RK4 stage at point slot pt with the stage's adjoint input
// mu = c1 v1 + c2 v2 (v2 may be NULL) and forward stage input u:
//   out = M^H mu + sum of w = -M mu + sum of w      (M^H = -M)
//   gradient shares += 2 Re(mu^H dM/dtheta u), theta = b (two terms), a, c.
// The three applications (M mu and the two b-derivative terms on u, the
// first of which also forms the a and c terms) share one k_apply launch.
int enqueue_reverse_stage(wpccc_plan_s* p, int pt, double z, const double2* v1, double c1, const double2* v2,
                          double c2, double2* out, std::initializer_list<const double2*> w, const double2* u,
                          hipStream_t st) {
    ApplyArgs a{};
    StageArgs& m = a.s[0];
    m = apply_args(p, pt, z, 0);
    m.u_in = v1;
    m.cu1 = c1;
    m.u_in2 = v2;
    m.cu2 = c2;
    m.alpha = -1.0;
    m.out = out;
    int k = 0;
    for (const double2* x : w) m.w[k++] = x;
    for (int d = 1; d <= 2; ++d) {
        StageArgs& g = a.s[d];
        g = apply_args(p, pt, z, d);
        g.u_in = u;
        g.dv = v1;
        g.cd1 = c1;
        g.dv2 = v2;
        g.cd2 = c2;
        g.grad = p->d_gpart;
        g.gslot = d - 1;
        if (d == 1) {
            g.model = 1;
            g.va = p->d_va;
            g.vc = p->d_vc;
        }
    }
    return launched(launch_apply(a, 3, p->c.meta, p->n_traj, p->stage_smem, p->apply_rows, p->gg, st), "k_apply");
}

// Capture one chunk of kChunkSteps steps for all paths on X into plan->gexec:
// the prologue reads its points from d_zall and the stages their step length
// from d_hall at the chunk index *d_chunk, which the last node advances.
int capture_chunk_graph(wpccc_plan_s* p, double2* X) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->gX = nullptr;
    if (!p->gstream) WPCCC_HIP_CHECK(hipStreamCreate(&p->gstream));
    WPCCC_HIP_CHECK(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeRelaxed));
    const bool timing = p->timer.on;
    p->timer.on = false;
    p->capturing = true;
    double dummy[kChunkPoints] = {0.0};
    int rc = enqueue_prologue(p, dummy, kChunkPoints, 0, p->n_traj, p->gstream);
    if (rc == WPCCC_OK) rc = enqueue_fpoint(p, 0, p->n_traj, 0, p->gstream);
    for (int i = 0; i < kChunkSteps && rc == WPCCC_OK; ++i) rc = enqueue_step(p, X, 0, p->n_traj, 2 * i, 0.0, p->gstream);
    if (rc == WPCCC_OK) rc = launched(launch_chunk_counter(p->d_chunk, 0, p->gstream), "k_chunk_counter");
    p->capturing = false;
    p->timer.on = timing;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gstream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    p->graph = g;
    WPCCC_HIP_CHECK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
    p->gX = X;
    return WPCCC_OK;
}

// Steps [0, n_full * kChunkSteps) of the grid by graph replays on st.
int propagate_graph(wpccc_plan_s* p, const double* zg, int n_full, double2* X, hipStream_t st) {
    if (n_full > p->g_cap) {
        if (p->g_copied) WPCCC_HIP_CHECK(hipEventSynchronize(p->g_copied));
        WPCCC_HIP_CHECK(hipStreamSynchronize(st));
        if (p->h_zh) (void)hipHostFree(p->h_zh);
        if (p->d_zall) (void)hipFree(p->d_zall);
        if (p->d_hall) (void)hipFree(p->d_hall);
        p->h_zh = nullptr;
        p->d_zall = p->d_hall = nullptr;
        p->g_cap = 0;
        // the graph reads the old arrays: capture again
        if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->gexec = nullptr;
        p->graph = nullptr;
        const size_t nz = (size_t)n_full * kChunkPoints, nh = (size_t)n_full * kChunkSteps;
        WPCCC_HIP_CHECK(hipHostMalloc((void**)&p->h_zh, (nz + nh) * sizeof(double), 0));
        int rc;
        if ((rc = dev_alloc(&p->d_zall, nz, p->bytes)) || (rc = dev_alloc(&p->d_hall, nh, p->bytes))) return rc;
        if (!p->d_chunk && (rc = dev_alloc(&p->d_chunk, 1, p->bytes))) return rc;
        if (!p->g_copied) WPCCC_HIP_CHECK(hipEventCreateWithFlags(&p->g_copied, hipEventDisableTiming));
        p->g_cap = n_full;
    }
    // the staging buffer may still feed the previous call's copy
    WPCCC_HIP_CHECK(hipEventSynchronize(p->g_copied));
    double* hz = p->h_zh;
    double* hh = p->h_zh + (size_t)p->g_cap * kChunkPoints;
    for (int c = 0; c < n_full; ++c)
        for (int i = 0; i <= kChunkSteps; ++i) {
            const int s = c * kChunkSteps + i;
            hz[(size_t)c * kChunkPoints + 2 * i] = zg[s];
            if (i < kChunkSteps) {
                hz[(size_t)c * kChunkPoints + 2 * i + 1] = 0.5 * (zg[s] + zg[s + 1]);
                hh[(size_t)c * kChunkSteps + i] = zg[s + 1] - zg[s];
            }
        }
    WPCCC_HIP_CHECK(hipMemcpyAsync(p->d_zall, hz, (size_t)n_full * kChunkPoints * sizeof(double),
                                   hipMemcpyHostToDevice, st));
    WPCCC_HIP_CHECK(hipMemcpyAsync(p->d_hall, hh, (size_t)n_full * kChunkSteps * sizeof(double),
                                   hipMemcpyHostToDevice, st));
    WPCCC_HIP_CHECK(hipEventRecord(p->g_copied, st));
    int rc;
    if (!p->gexec || p->gX != X) {
        // the capture stream must not run ahead of work already queued on st
        WPCCC_HIP_CHECK(hipStreamSynchronize(st));
        if ((rc = capture_chunk_graph(p, X))) return rc;
    }
    if ((rc = launched(launch_chunk_counter(p->d_chunk, 1, st), "k_chunk_counter"))) return rc;
    for (int c = 0; c < n_full; ++c) WPCCC_HIP_CHECK(hipGraphLaunch(p->gexec, st));
    return WPCCC_OK;
}

// Stage configuration of a one-centre plan: rows per workgroup and launch
// form (kernel by kernel, or the persistent k_chunk where its grid fits on
// the device at once).  Each admissible candidate runs kTuneSteps RK4 steps
// over the plan's launch batch from zero amplitudes (the table and state
// traffic of a real step), once to warm up and kTunePasses times timed; the
// candidate with the fastest pass is kept.
constexpr int kTuneSteps = 8;
constexpr double kAdjointStoreAll = 256.0 * (1 << 20);  // bytes of stored states and stage inputs below which nothing is recomputed
constexpr int kTunePasses = 3;

int tune_stage(wpccc_plan_s* p, const int* cand, int n_cand, int launch_req, hipStream_t st) {
    const Meta& m = p->c.meta;
    const int nj = p->batched ? p->n_traj : 1;
    const size_t V = (size_t)p->n_traj * p->n_pad * sizeof(double2);
    double2* X = nullptr;
    long long scratch_bytes = 0;
    int rc = dev_alloc(&X, (size_t)p->n_traj * p->n_pad, scratch_bytes);
    if (rc) return rc;
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    hipError_t e = hipMemsetAsync(X, 0, V, st);
    for (double2* q : {p->d_Ua, p->d_Ub, p->d_Xacc})
        if (e == hipSuccess) e = hipMemsetAsync(q, 0, V, st);
    if (e == hipSuccess) e = hipEventCreate(&ev.e0);
    if (e == hipSuccess) e = hipEventCreate(&ev.e1);
    if (e != hipSuccess) {
        (void)hipFree(X);
        set_error("stage tuning failed: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    double pts[2 * kTuneSteps + 1], hs[kTuneSteps];
    for (int i = 0; i <= 2 * kTuneSteps; ++i) pts[i] = 0.37 + 0.005 * i;  // b > 0, so R > 0 at any z
    for (int i = 0; i < kTuneSteps; ++i) hs[i] = 0.01;
    rc = enqueue_prologue(p, pts, 2 * kTuneSteps + 1, 0, nj, st);
    const bool timing = p->timer.on;
    p->timer.on = false;
    float best_ms = 1e30f;
    int best_rows = 0, best_launch = 0;
    const int saved_rows = p->stage_rows, saved_smem = p->stage_smem_rows;
    const bool direct_ok = !p->interp && !p->gg && p->cache_req != WPCCC_CACHE_ON;
    const bool cache_ok = p->cache_req != WPCCC_CACHE_OFF;
    bool best_cache = cache_ok;
    auto time_it = [&](int rows, int launch, bool cache, float* ms) -> int {
        const int smem = stage_smem_bytes(m, rows, p->gg);
        p->stage_rows = rows;
        p->stage_smem_rows = smem;
        p->fcache = cache;
        // a warm-up pass, then the fastest of kTunePasses timed passes
        int r = WPCCC_OK;
        *ms = 1e30f;
        for (int pass = 0; pass <= kTunePasses && r == WPCCC_OK; ++pass) {
            if (pass > 0 && hipEventRecord(ev.e0, st) != hipSuccess) r = WPCCC_EHIP;
            if (launch == WPCCC_LAUNCH_PERSISTENT) {
                if (r == WPCCC_OK) r = enqueue_chunk(p, X, 0, nj, hs, kTuneSteps, rows, chunk_smem_bytes(m, rows), st);
            } else {
                if (r == WPCCC_OK) r = enqueue_fpoint(p, 0, nj, 0, st);
                for (int i = 0; i < kTuneSteps && r == WPCCC_OK; ++i) r = enqueue_step(p, X, 0, nj, 2 * i, hs[i], st);
            }
            float t = 0.f;
            if (pass > 0 && r == WPCCC_OK &&
                (hipEventRecord(ev.e1, st) != hipSuccess || hipEventSynchronize(ev.e1) != hipSuccess ||
                 hipEventElapsedTime(&t, ev.e0, ev.e1) != hipSuccess)) {
                set_error("stage tuning failed: %s", hipGetErrorString(hipGetLastError()));
                r = WPCCC_EHIP;
            }
            if (pass > 0 && r == WPCCC_OK) *ms = std::min(*ms, t);
        }
        return r;
    };
    for (int ci = 0; ci < n_cand && rc == WPCCC_OK; ++ci) {
        const int rows = cand[ci];
        const int smem = stage_smem_bytes(m, rows, p->gg);
        if (smem > kMaxDynLds || !stage_rows_fit(m, rows)) continue;
        for (int launch : {WPCCC_LAUNCH_STAGES, WPCCC_LAUNCH_PERSISTENT}) {
            if (launch_req != WPCCC_LAUNCH_AUTO && launch != launch_req) continue;
            if (launch == WPCCC_LAUNCH_PERSISTENT && (p->mixed || p->interp || p->gg)) continue;
            if (launch == WPCCC_LAUNCH_PERSISTENT &&
                (chunk_smem_bytes(m, rows) > kMaxDynLds || !chunk_fits(m, nj, rows, chunk_smem_bytes(m, rows))))
                continue;
            for (int cache = 1; cache >= 0; --cache) {
                if (!cache && (launch == WPCCC_LAUNCH_PERSISTENT || !direct_ok)) continue;
                if (cache && !cache_ok && launch != WPCCC_LAUNCH_PERSISTENT) continue;
                float ms = 0.f;
                if ((rc = time_it(rows, launch, cache != 0, &ms))) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best_rows = rows;
                    best_launch = launch;
                    best_cache = cache != 0;
                }
            }
            if (rc) break;
        }
    }
    p->fcache = best_cache;
    p->timer.on = timing;
    const hipError_t es = hipStreamSynchronize(st);
    (void)hipFree(X);
    if (rc == WPCCC_OK && es != hipSuccess) {
        set_error("stage tuning failed: %s", hipGetErrorString(es));
        rc = WPCCC_EHIP;
    }
    if (rc) return rc;
    if (!best_rows) {
        p->stage_rows = saved_rows;
        p->stage_smem_rows = saved_smem;
        set_error("wpccc_plan_create: the persistent stage kernel's grid does not fit on the device at once");
        return WPCCC_ENOTSUP;
    }
    p->stage_rows = best_rows;
    p->stage_smem_rows = stage_smem_bytes(m, best_rows, p->gg);
    p->chunk_smem = chunk_smem_bytes(m, best_rows);
    p->launch = best_launch;
    return WPCCC_OK;
}

// Channel code of state i of a basis with energies eps (kChElastic .. kChProjCont).
unsigned char channel_code(const std::vector<double>& eps, int i, bool projectile) {
    if (projectile) return eps[i] < 0.0 ? kChCapture : kChProjCont;
    if (i == 0) return kChElastic;
    return eps[i] < 0.0 ? kChExcitation : kChTargetCont;
}

// Observable tables of a plan: the states of path j are the target basis of
// its set (and the projectile basis after it, two-centre); group = (set, v).
int build_observables(wpccc_plan_s* p, int n_traj, int n_pad, const std::vector<const HostBasis*>& tb,
                      const std::vector<const HostBasis*>& pb, const int* set_of, const double* b, const double* v) {
    std::vector<unsigned char> codes((size_t)n_traj * n_pad, kChPadding);
    std::vector<int> group_of(n_traj);
    std::vector<std::pair<int, double>> keys;
    for (int j = 0; j < n_traj; ++j) {
        const int s = set_of ? set_of[j] : 0;
        unsigned char* c = codes.data() + (size_t)j * n_pad;
        const HostBasis& t = *tb[s];
        for (int i = 0; i < t.n_states; ++i) c[i] = channel_code(t.eps, i, false);
        if (!pb.empty())
            for (int i = 0; i < pb[s]->n_states; ++i) c[t.n_states + i] = channel_code(pb[s]->eps, i, true);
        const std::pair<int, double> key(s, v[j]);
        int g = 0;
        while (g < (int)keys.size() && keys[g] != key) ++g;
        if (g == (int)keys.size()) keys.push_back(key);
        group_of[j] = g;
    }
    const int rc = obs_build(p->obs, n_traj, n_pad, codes, group_of, std::vector<double>(b, b + n_traj));
    if (rc == WPCCC_OK) p->bytes += p->obs.bytes;
    return rc;
}

}  // namespace

#define TRY(x)                 \
    do {                       \
        int rc_ = (x);         \
        if (rc_ != WPCCC_OK) { \
            free_plan(plan);   \
            return rc_;        \
        }                      \
    } while (0)

extern "C" {

const char* wpccc_last_error(void) { return g_err.c_str(); }

int wpccc_measure_mfma(double* tflops_f64, double* tflops_f32, void* stream) {
    clear_error();
    const hipError_t e = measure_mfma(tflops_f64, tflops_f32, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_error("wpccc_measure_mfma: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

int wpccc_zgesv_batched(int n, int batch, const void* A_dev, const void* B_dev, void* X_dev, void* stream) {
    clear_error();
    return lu_solve_batched(n, batch, A_dev, B_dev, X_dev, (hipStream_t)stream);
}

const char* wpccc_version(void) { return "0.3.0"; }

int wpccc_basis(const wpccc_basis_spec* spec, wpccc_basis_t* out) {
    clear_error();
    if (!spec || !out) {
        set_error("wpccc_basis: NULL argument");
        return WPCCC_EINVAL;
    }
    *out = nullptr;
    wpccc_basis_s* b = new (std::nothrow) wpccc_basis_s;
    if (!b) {
        set_error("wpccc_basis: out of host memory");
        return WPCCC_ENOMEM;
    }
    int rc;
    try {
        rc = build_host_basis(*spec, b->hb);
    } catch (const std::bad_alloc&) {
        set_error("wpccc_basis: out of host memory");
        rc = WPCCC_ENOMEM;
    }
    if (rc != WPCCC_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return WPCCC_OK;
}

int wpccc_basis_info(wpccc_basis_t basis, int* n_states, int* n_radial, int* n_r) {
    if (!basis) {
        set_error("wpccc_basis_info: NULL basis");
        return WPCCC_EINVAL;
    }
    if (n_states) *n_states = basis->hb.n_states;
    if (n_radial) *n_radial = basis->hb.n_f;
    if (n_r) *n_r = basis->hb.n_r;
    return WPCCC_OK;
}

int wpccc_basis_export(wpccc_basis_t basis, double* r_host, double* w_host, double* phi_host,
                       double* eps_host, int* lmi_host) {
    if (!basis) {
        set_error("wpccc_basis_export: NULL basis");
        return WPCCC_EINVAL;
    }
    const HostBasis& hb = basis->hb;
    if (r_host) std::memcpy(r_host, hb.r.data(), hb.r.size() * sizeof(double));
    if (w_host) std::memcpy(w_host, hb.w.data(), hb.w.size() * sizeof(double));
    if (phi_host) std::memcpy(phi_host, hb.phi.data(), hb.phi.size() * sizeof(double));
    if (eps_host) std::memcpy(eps_host, hb.eps.data(), hb.eps.size() * sizeof(double));
    if (lmi_host)
        for (int s = 0; s < hb.n_states; ++s) {
            lmi_host[3 * s] = hb.st_l[s];
            lmi_host[3 * s + 1] = hb.st_m[s];
            lmi_host[3 * s + 2] = hb.st_i[s];
        }
    return WPCCC_OK;
}

int wpccc_basis_destroy(wpccc_basis_t basis) {
    delete basis;
    return WPCCC_OK;
}

int wpccc_plan_create(wpccc_basis_t target, int n_traj, const double* b_host, const double* v_host,
                      const wpccc_plan_opts* opts, void* stream, wpccc_plan_t* out) {
    clear_error();
    if (!target || !b_host || !v_host || !out || n_traj < 1) {
        set_error("wpccc_plan_create: NULL argument or n_traj < 1");
        return WPCCC_EINVAL;
    }
    *out = nullptr;
    wpccc_plan_opts o{};
    o.Zp = 1.0;
    o.batched = 1;
    if (opts) o = *opts;
    if (o.Zp == 0.0) o.Zp = 1.0;
    if (o.two_centre) {
        set_error("wpccc_plan_create: use wpccc_plan_create_2c for the two-centre form");
        return WPCCC_EINVAL;
    }
    if (o.precision != WPCCC_FP64 && o.precision != WPCCC_MIXED) {
        set_error("wpccc_plan_create: precision must be WPCCC_FP64 or WPCCC_MIXED");
        return WPCCC_EINVAL;
    }
    const bool mixed = o.precision == WPCCC_MIXED;
    if (mixed && o.stage_launch == WPCCC_LAUNCH_PERSISTENT) {
        set_error("wpccc_plan_create: the persistent stage kernel has no reduced-precision form");
        return WPCCC_ENOTSUP;
    }
    if (o.batched != 0 && o.batched != 1) {
        set_error("wpccc_plan_create: batched must be 0 or 1");
        return WPCCC_EINVAL;
    }
    if (o.solve != 0 || o.symmetric != 0) {
        set_error("wpccc_plan_create: solve and symmetric are two-centre options (the one-centre form has S = I)");
        return WPCCC_EINVAL;
    }
    if (o.radial != WPCCC_RADIAL_EXACT && o.radial != WPCCC_RADIAL_INTERP) {
        set_error("wpccc_plan_create: radial must be WPCCC_RADIAL_EXACT or WPCCC_RADIAL_INTERP");
        return WPCCC_EINVAL;
    }
    const bool interp = o.radial == WPCCC_RADIAL_INTERP;
    if (o.stage_cache < WPCCC_CACHE_AUTO || o.stage_cache > WPCCC_CACHE_OFF) {
        set_error("wpccc_plan_create: stage_cache must be WPCCC_CACHE_AUTO, _ON or _OFF");
        return WPCCC_EINVAL;
    }
    if (o.stage_cache == WPCCC_CACHE_OFF && interp) {
        set_error("wpccc_plan_create: the interpolated form needs the radial-integral cache");
        return WPCCC_ENOTSUP;
    }
    if (interp && (mixed || o.stage_launch == WPCCC_LAUNCH_PERSISTENT)) {
        set_error("wpccc_plan_create: the interpolated radial integrals are an FP64, one-launch-per-stage form");
        return WPCCC_ENOTSUP;
    }
    for (int j = 0; j < n_traj; ++j)
        if (!(b_host[j] > 0.0) || !(v_host[j] > 0.0) || !std::isfinite(b_host[j]) || !std::isfinite(v_host[j])) {
            set_error("wpccc_plan_create: path %d needs finite b > 0 and v > 0", j);
            return WPCCC_EINVAL;
        }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("wpccc_plan_create: no HIP device available");
        return WPCCC_EHIP;
    }
    const HostBasis& hb = target->hb;
    wpccc_plan_s* plan = new (std::nothrow) wpccc_plan_s;
    if (!plan) {
        set_error("wpccc_plan_create: out of host memory");
        return WPCCC_ENOMEM;
    }
    hipStream_t st = (hipStream_t)stream;
    plan->n_traj = n_traj;
    plan->batched = o.batched ? 1 : 0;
    plan->Zp = o.Zp;
    plan->b.assign(b_host, b_host + n_traj);
    plan->v.assign(v_host, v_host + n_traj);
    const int N = hb.n_states;
    plan->n_pad = (N + 7) & ~7;
    plan->mixed = mixed;
    plan->interp = interp;
    plan->cache_req = o.stage_cache;
    plan->fcache = o.stage_cache != WPCCC_CACHE_OFF;
    TRY(centre_build(hb, st, plan->c, o.model_a, o.model_c, o.Zp,
                     interp ? kRadialInterp : (mixed ? kRadialMoments32 : kRadialMoments)));
    plan->ckpt_every = o.checkpoint_every;
    plan->use_graph = o.graph != 0;
    const Meta& m = plan->c.meta;
    plan->stage_smem = stage_smem_bytes(m);
    // the large-basis form when no regular tiling fits the LDS
    bool regular_fits = false;
    for (int r : kStageRowsList)
        regular_fits = regular_fits || (stage_smem_bytes(m, r) <= kMaxDynLds && stage_rows_fit(m, r));
    plan->gg = !regular_fits;
    if (plan->gg && o.stage_cache == WPCCC_CACHE_OFF) {
        set_error("wpccc_plan_create: a basis this large needs the radial-integral cache");
        free_plan(plan);
        return WPCCC_ENOTSUP;
    }
    if (plan->gg && o.stage_launch == WPCCC_LAUNCH_PERSISTENT) {
        set_error("wpccc_plan_create: the persistent stage kernel does not take a basis this large");
        free_plan(plan);
        return WPCCC_ENOTSUP;
    }
    bool rows_ok = o.stage_rows == 0;
    for (int r : kStageRowsList) rows_ok = rows_ok || (!plan->gg && o.stage_rows == r);
    for (int r : kStageRowsGG) rows_ok = rows_ok || (plan->gg && o.stage_rows == r);
    if (!rows_ok) {
        set_error(plan->gg ? "wpccc_plan_create: stage_rows must be 0, 1, 2 or 4 for a basis this large"
                           : "wpccc_plan_create: stage_rows must be 0, 4, 5, 6, 7, 8, 10, 12 or 16");
        free_plan(plan);
        return plan->gg && o.stage_rows > 0 ? WPCCC_ENOTSUP : WPCCC_EINVAL;
    }
    if (o.stage_launch < WPCCC_LAUNCH_AUTO || o.stage_launch > WPCCC_LAUNCH_PERSISTENT) {
        set_error("wpccc_plan_create: stage_launch must be WPCCC_LAUNCH_AUTO, _STAGES or _PERSISTENT");
        free_plan(plan);
        return WPCCC_EINVAL;
    }
    // untimed default tiling: kRowsPerBlock rows, or the largest admissible
    // smaller tiling whose LDS fits (large bases)
    int rows0 = o.stage_rows;
    if (!rows0 && plan->gg) {
        rows0 = kStageRowsGG[0];
        for (int r : kStageRowsGG)
            if (stage_smem_bytes(m, r, true) <= kMaxDynLds && stage_rows_fit(m, r)) rows0 = r;
    } else if (!rows0) {
        rows0 = kRowsPerBlock;
        if (stage_smem_bytes(m, rows0) > kMaxDynLds)
            for (int r : kStageRowsList)
                if (r < kRowsPerBlock && stage_smem_bytes(m, r) <= kMaxDynLds) rows0 = r;
    }
    plan->stage_rows = rows0;
    plan->stage_smem_rows = stage_smem_bytes(m, plan->stage_rows, plan->gg);
    if (!stage_rows_fit(m, plan->stage_rows)) {
        set_error("wpccc_plan_create: stage_rows %d is too many for l_max = %d (rows x (2 l_max + 1) must not "
                  "exceed %d)", plan->stage_rows, m.l_max, kStageThreads);
        free_plan(plan);
        return WPCCC_EINVAL;
    }
    if (plan->stage_smem_rows > kMaxDynLds) {
        set_error("wpccc_plan_create: basis too large for the stage kernel's LDS (%d bytes at %d rows%s)",
                  plan->stage_smem_rows, plan->stage_rows, plan->gg ? ", angular factors in global memory" : "");
        free_plan(plan);
        return WPCCC_ENOTSUP;
    }
    // the adjoint's operator kernel (k_apply): kRowsPerBlock rows, or
    // kApplyRowsLarge where those do not fit the LDS; with the large-basis
    // form 4, 2 or 1 rows
    plan->apply_ok = false;
    for (int r : plan->gg ? std::initializer_list<int>{4, 2, 1}
                          : std::initializer_list<int>{kRowsPerBlock, kApplyRowsLarge})
        if (!plan->apply_ok && stage_smem_bytes(m, r, plan->gg) <= kMaxDynLds && stage_rows_fit(m, r)) {
            plan->apply_ok = true;
            plan->apply_rows = r;
            plan->stage_smem = stage_smem_bytes(m, r, plan->gg);
        }
    long long& tot = plan->bytes;
    tot = plan->c.bytes;
    TRY(dev_alloc(&plan->d_b, (size_t)n_traj, tot));
    TRY(dev_alloc(&plan->d_v, (size_t)n_traj, tot));
    TRY(dev_alloc(&plan->d_flag, 1, tot));
    TRY(dev_alloc(&plan->d_bar, (size_t)n_traj * kBarStride, tot));
    TRY(dev_alloc(&plan->d_gpart, (size_t)n_traj * kGradSlots * stage_chunks(m, plan->apply_rows), tot));
    std::vector<StageTile> tiles;
    for (int i = 0; i < kNumStageRows; ++i) {
        std::vector<StageTile> t;
        stage_tiles(m, kStageRowsList[i], t);
        plan->tile_off[i] = (int)tiles.size();
        plan->tile_n[i] = (int)t.size();
        tiles.insert(tiles.end(), t.begin(), t.end());
    }
    for (int i = 0; i < 3; ++i) {
        std::vector<StageTile> t;
        stage_tiles(m, kStageRowsGG[i], t);
        plan->tile_off_gg[i] = (int)tiles.size();
        plan->tile_n_gg[i] = (int)t.size();
        tiles.insert(tiles.end(), t.begin(), t.end());
    }
    {
        // resident workgroups of the device for each tiling (0 if unknown:
        // then the tiles are only balanced in size)
        int dev = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            n_cu = 0;
        }
        const int n_launch = plan->batched ? n_traj : 1;
        for (int i = 0; i < kNumStageRows; ++i) {
            const int r = kStageRowsList[i];
            const long long slots = (long long)n_cu * stage_wgs_per_cu(r, stage_smem_bytes(m, r));
            std::vector<StageTile> t;
            stage_tiles_balanced(m, r, n_launch, slots, t);
            plan->tile_off_bal[i] = (int)tiles.size();
            plan->tile_n_bal[i] = (int)t.size();
            tiles.insert(tiles.end(), t.begin(), t.end());
        }
    }
    TRY(dev_alloc(&plan->d_tiles, tiles.size(), tot));
    TRY(dev_alloc(&plan->d_Frow1, (size_t)m.n_frow, tot));
    TRY(dev_alloc(&plan->d_G1, (size_t)m.n_g, tot));
    TRY(dev_alloc(&plan->d_PH1, (size_t)N, tot));
    TRY(dev_alloc(&plan->d_Ua, (size_t)n_traj * plan->n_pad, tot));
    TRY(dev_alloc(&plan->d_Ub, (size_t)n_traj * plan->n_pad, tot));
    TRY(dev_alloc(&plan->d_Xacc, (size_t)n_traj * plan->n_pad, tot));
    TRY(dev_alloc(&plan->d_kidx, (size_t)n_traj * kChunkPoints, tot));
    TRY(dev_alloc(&plan->d_rpow, (size_t)n_traj * kChunkPoints * kRpow, tot));
    TRY(dev_alloc(&plan->d_pbar, (size_t)n_traj * kChunkPoints * kMaxPb, tot));
    TRY(dev_alloc(&plan->d_ph, (size_t)n_traj * kChunkPoints * m.n_f, tot));
    TRY(dev_alloc_bytes(&plan->d_fc, (size_t)kFcSlots * n_traj * m.n_frow * (mixed ? sizeof(float) : sizeof(double)),
                        tot));
    std::vector<double> va, vc;
    model_blocks(hb, o.model_a, o.model_c, va, vc);
    TRY(dev_alloc(&plan->d_va, va.size(), tot));
    TRY(dev_alloc(&plan->d_vc, vc.size(), tot));
    hipError_t e = hipMemcpyAsync(plan->d_b, b_host, (size_t)n_traj * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->d_v, v_host, (size_t)n_traj * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(plan->d_flag, 0, sizeof(int), st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->d_tiles, tiles.data(), tiles.size() * sizeof(StageTile), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->d_va, va.data(), va.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(plan->d_vc, vc.data(), vc.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const int smem16 = chunk_smem_bytes(m, 16);
    const int smem_max = std::min(kMaxDynLds, std::max(smem16, plan->stage_smem));
    if (e == hipSuccess && smem_max > 64 * 1024) e = stage_set_smem_limit(m.l_max, smem_max);
    if (e != hipSuccess) {
        set_error("wpccc_plan_create: device setup failed: %s", hipGetErrorString(e));
        free_plan(plan);
        return WPCCC_EHIP;
    }
    if (o.stage_rows == 0 || o.stage_launch == WPCCC_LAUNCH_AUTO) {
        const int* cand = o.stage_rows ? &o.stage_rows : (plan->gg ? kStageRowsGG : kStageRowsList);
        TRY(tune_stage(plan, cand, o.stage_rows ? 1 : (plan->gg ? 3 : kNumStageRows), o.stage_launch, st));
    } else if (o.stage_launch == WPCCC_LAUNCH_PERSISTENT) {
        // nothing to choose: check that the grid can be resident at once
        const int nj = plan->batched ? n_traj : 1;
        plan->chunk_smem = chunk_smem_bytes(m, plan->stage_rows);
        if (plan->chunk_smem > kMaxDynLds || !chunk_fits(m, nj, plan->stage_rows, plan->chunk_smem)) {
            set_error("wpccc_plan_create: the persistent stage kernel's grid does not fit on the device at once");
            free_plan(plan);
            return WPCCC_ENOTSUP;
        }
        plan->launch = WPCCC_LAUNCH_PERSISTENT;
    }
    TRY(build_observables(plan, n_traj, plan->n_pad, {&hb}, {}, nullptr, b_host, v_host));
    *out = plan;
    return WPCCC_OK;
}

int wpccc_plan_create_2c(const wpccc_basis_t* targets, const wpccc_basis_t* projectiles, int n_sets, int n_traj,
                         const int* set_of_traj, const double* b_host, const double* v_host,
                         const wpccc_plan_opts* opts, void* stream, wpccc_plan_t* out) {
    clear_error();
    if (!targets || !projectiles || n_sets < 1 || n_traj < 1 || !set_of_traj || !b_host || !v_host || !out) {
        set_error("wpccc_plan_create_2c: NULL argument or empty plan");
        return WPCCC_EINVAL;
    }
    *out = nullptr;
    wpccc_plan_opts o{};
    o.batched = 1;
    if (opts) o = *opts;
    o.two_centre = 1;
    if (o.n_eta == 0) o.n_eta = 256;
    if (o.n_tau == 0) o.n_tau = 512;
    wpccc_plan_s* plan = new (std::nothrow) wpccc_plan_s;
    if (!plan) {
        set_error("wpccc_plan_create_2c: out of host memory");
        return WPCCC_ENOMEM;
    }
    const int rc = plan2c_create(targets, projectiles, n_sets, n_traj, set_of_traj, b_host, v_host, o,
                                 &plan->timer, (hipStream_t)stream, &plan->p2c);
    if (rc != WPCCC_OK) {
        plan->p2c = nullptr;
        free_plan(plan);
        return rc;
    }
    std::vector<const HostBasis*> tb, pb;
    for (int s = 0; s < n_sets; ++s) {
        tb.push_back(&targets[s]->hb);
        pb.push_back(&projectiles[s]->hb);
    }
    int n_pad = 0;
    plan2c_info(plan->p2c, nullptr, nullptr, &n_pad, nullptr);
    TRY(build_observables(plan, n_traj, n_pad, tb, pb, set_of_traj, b_host, v_host));
    *out = plan;
    return WPCCC_OK;
}

int wpccc_plan_info(wpccc_plan_t plan, int* n_traj, int* n_states, int* n_pad, long long* device_bytes) {
    if (!plan) {
        set_error("wpccc_plan_info: NULL plan");
        return WPCCC_EINVAL;
    }
    if (plan->p2c) return plan2c_info(plan->p2c, n_traj, n_states, n_pad, device_bytes);
    if (n_traj) *n_traj = plan->n_traj;
    if (n_states) *n_states = plan->c.meta.n_states;
    if (n_pad) *n_pad = plan->n_pad;
    if (device_bytes) *device_bytes = plan->bytes;
    return WPCCC_OK;
}

int wpccc_plan_path_info(wpccc_plan_t plan, int j, int* n_states, int* n_target) {
    if (!plan) {
        set_error("wpccc_plan_path_info: NULL plan");
        return WPCCC_EINVAL;
    }
    if (plan->p2c) return plan2c_path_info(plan->p2c, j, n_states, n_target);
    if (j < 0 || j >= plan->n_traj) {
        set_error("wpccc_plan_path_info: path index out of range");
        return WPCCC_EINVAL;
    }
    if (n_states) *n_states = plan->c.meta.n_states;
    if (n_target) *n_target = plan->c.meta.n_states;
    return WPCCC_OK;
}

int wpccc_plan_stage_rows(wpccc_plan_t plan, int* rows) {
    if (!plan || !rows) {
        set_error("wpccc_plan_stage_rows: NULL argument");
        return WPCCC_EINVAL;
    }
    *rows = plan->p2c ? 0 : plan->stage_rows;
    return WPCCC_OK;
}

int wpccc_plan_stage_cache(wpccc_plan_t plan, int* cached) {
    if (!plan || !cached) {
        set_error("wpccc_plan_stage_cache: NULL argument");
        return WPCCC_EINVAL;
    }
    *cached = (!plan->p2c && plan->fcache) ? 1 : 0;
    return WPCCC_OK;
}

int wpccc_plan_stage_launch(wpccc_plan_t plan, int* launch) {
    if (!plan || !launch) {
        set_error("wpccc_plan_stage_launch: NULL argument");
        return WPCCC_EINVAL;
    }
    *launch = plan->p2c ? WPCCC_LAUNCH_STAGES : plan->launch;
    return WPCCC_OK;
}

int wpccc_plan_destroy(wpccc_plan_t plan) {
    if (plan) (void)hipDeviceSynchronize();
    free_plan(plan);
    return WPCCC_OK;
}

int wpccc_plan_status(wpccc_plan_t plan, void* stream) {
    if (!plan) {
        set_error("wpccc_plan_status: NULL plan");
        return WPCCC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (plan->p2c) return plan2c_status(plan->p2c, st);
    int flag = 0;
    WPCCC_HIP_CHECK(hipMemcpyAsync(&flag, plan->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    WPCCC_HIP_CHECK(hipMemsetAsync(plan->d_flag, 0, sizeof(int), st));
    if (flag & 2) {
        set_error("a path barrier of the persistent stage kernel timed out (results are incomplete)");
        return WPCCC_EHIP;
    }
    if (flag) {
        set_error("non-finite amplitude detected during propagation");
        return WPCCC_ENUMERIC;
    }
    return WPCCC_OK;
}

}  // extern "C"

// Device scratch of wpccc_couplings_noalloc: the radial integrals, angular
// factors and phases of one path at one point, each part starting on a
// 256-byte boundary.  Each GPU the library runs on holds its own copy for the
// life of the process; host code uses only the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

// Argument checks shared by wpccc_couplings and wpccc_couplings_noalloc for a
// one-centre plan.
int couplings_1c_check(const char* fn, wpccc_plan_t plan, int j, double z, void* S_dev) {
    if (j < 0 || j >= plan->n_traj) {
        set_error("%s: path index out of range", fn);
        return WPCCC_EINVAL;
    }
    if (S_dev) {
        set_error("%s: S_dev must be NULL for a one-centre plan", fn);
        return WPCCC_EINVAL;
    }
    if (!(std::sqrt(plan->b[j] * plan->b[j] + z * z) > 0.0)) {
        set_error("%s: R = 0", fn);
        return WPCCC_EINVAL;
    }
    return WPCCC_OK;
}

// Dense one-centre couplings of path j at z: k_slot_setup fills the radial
// integrals Frow, the angular factors G and the phases PH of the point (every
// element is written), k_couplings_dense combines them into H.
int couplings_1c(wpccc_plan_t plan, int j, double z, double* Frow, double* G, double2* PH, void* H_dev,
                 hipStream_t st) {
    const Meta& m = plan->c.meta;
    SetupArgs a;
    a.meta = plan->c.d_meta;
    a.tb = plan->tables();
    a.z = z;
    a.j = j;
    a.Frow = Frow;
    a.G = G;
    a.PH = PH;
    a.nbF = (m.n_frow + 255) / 256;
    a.nbP = (m.n_states + 255) / 256;
    hipError_t e = launch_slot_setup(a, m, st, plan->timer.open(kSetup));
    int rc = launched(e, "k_slot_setup");
    if (rc) return rc;
    e = launch_couplings_dense(plan->c.d_meta, m, Frow, G, PH, plan->Zp, (double2*)H_dev, st,
                               plan->timer.open(kDense));
    return launched(e, "k_couplings_dense");
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void** out) {
    int dev = 0;
    WPCCC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("wpccc_couplings_noalloc: device ordinal %d beyond the library's %d", dev, kMaxDevices);
        return WPCCC_ENOTSUP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("wpccc_couplings_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                      hipGetErrorString(e));
            return WPCCC_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return WPCCC_OK;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

extern "C" {

int wpccc_couplings(wpccc_plan_t plan, int j, double z, void* H_dev, void* S_dev, void* stream) {
    clear_error();
    if (!plan || !H_dev || !std::isfinite(z)) {
        set_error("wpccc_couplings: bad plan, H_dev or z");
        return WPCCC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (plan->p2c) return plan2c_couplings(plan->p2c, j, z, H_dev, S_dev, st);
    const int rc = couplings_1c_check("wpccc_couplings", plan, j, z, S_dev);
    if (rc) return rc;
    return couplings_1c(plan, j, z, plan->d_Frow1, plan->d_G1, plan->d_PH1, H_dev, st);
}

int wpccc_couplings_noalloc(wpccc_plan_t plan, int j, double z, void* H_dev, void* S_dev, void* stream) {
    clear_error();
    if (!plan || !H_dev || !std::isfinite(z)) {
        set_error("wpccc_couplings_noalloc: bad plan, H_dev or z");
        return WPCCC_EINVAL;
    }
    if (plan->p2c) {
        set_error("wpccc_couplings_noalloc: one-centre plans only");
        return WPCCC_ENOTSUP;
    }
    int rc = couplings_1c_check("wpccc_couplings_noalloc", plan, j, z, S_dev);
    if (rc) return rc;
    const Meta& m = plan->c.meta;
    const size_t nF = align256((size_t)m.n_frow * sizeof(double));
    const size_t nG = align256((size_t)m.n_g * sizeof(double));
    const size_t need = nF + nG + align256((size_t)m.n_states * sizeof(double2));
    if (need > kNoAllocScratchBytes) {
        set_error("wpccc_couplings_noalloc: the basis needs %zu bytes of scratch, more than the %zu the "
                  "library holds per device", need, kNoAllocScratchBytes);
        return WPCCC_ENOTSUP;
    }
    void* base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    char* s = static_cast<char*>(base);
    return couplings_1c(plan, j, z, reinterpret_cast<double*>(s), reinterpret_cast<double*>(s + nF),
                        reinterpret_cast<double2*>(s + nF + nG), H_dev, (hipStream_t)stream);
}

int wpccc_step(wpccc_plan_t plan, void* X_dev, double z, double h, void* stream) {
    clear_error();
    if (!plan || !X_dev || !(h != 0.0) || !std::isfinite(z) || !std::isfinite(h)) {
        set_error("wpccc_step: bad plan, X_dev, z or h");
        return WPCCC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    if (plan->p2c) return plan2c_step(plan->p2c, X_dev, z, h, st);
    if (path_hits_origin(plan, z) || path_hits_origin(plan, z + 0.5 * h) || path_hits_origin(plan, z + h)) {
        set_error("wpccc_step: R = 0 on the step");
        return WPCCC_EINVAL;
    }
    double2* X = (double2*)X_dev;
    const int chunk = plan->batched ? plan->n_traj : 1;
    for (int j0 = 0; j0 < plan->n_traj; j0 += chunk) {
        const int nj = std::min(chunk, plan->n_traj - j0);
        const double pts[3] = {z, z + 0.5 * h, z + h};
        int rc = enqueue_prologue(plan, pts, 3, j0, nj, st);
        if (rc) return rc;
        if ((rc = enqueue_fpoint(plan, j0, nj, 0, st))) return rc;
        if ((rc = enqueue_step(plan, X, j0, nj, 0, h, st))) return rc;
    }
    return WPCCC_OK;
}

int wpccc_propagate(wpccc_plan_t plan, const double* zgrid_host, int n_points, void* X_dev, void* P_dev,
                    void* norm_dev, void* stream) {
    clear_error();
    if (!plan || !X_dev) {
        set_error("wpccc_propagate: bad plan or X_dev");
        return WPCCC_EINVAL;
    }
    int rc = check_grid(zgrid_host, n_points);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (plan->p2c) return plan2c_propagate(plan->p2c, zgrid_host, n_points, X_dev, P_dev, norm_dev, st);
    for (int i = 0; i < n_points; ++i)
        if (path_hits_origin(plan, zgrid_host[i]) ||
            (i + 1 < n_points && path_hits_origin(plan, 0.5 * (zgrid_host[i] + zgrid_host[i + 1])))) {
            set_error("wpccc_propagate: R = 0 on the grid");
            return WPCCC_EINVAL;
        }
    double2* X = (double2*)X_dev;
    const int chunk = plan->batched ? plan->n_traj : 1;
    int first = 0;  // first grid point of the kernel-by-kernel part
    if (plan->use_graph && plan->batched && (n_points - 1) >= kChunkSteps) {
        const int n_full = (n_points - 1) / kChunkSteps;
        if ((rc = propagate_graph(plan, zgrid_host, n_full, X, st))) return rc;
        first = n_full * kChunkSteps;
    }
    for (int j0 = 0; j0 < plan->n_traj; j0 += chunk) {
        const int nj = std::min(chunk, plan->n_traj - j0);
        // chunks of at most kChunkSteps steps share one prologue launch:
        // point 2i is zgrid[c0+i], point 2i+1 the midpoint of step c0+i
        for (int c0 = first; c0 + 1 < n_points; c0 += kChunkSteps) {
            const int ns = std::min(kChunkSteps, n_points - 1 - c0);
            double pts[kChunkPoints];
            for (int i = 0; i <= ns; ++i) {
                pts[2 * i] = zgrid_host[c0 + i];
                if (i < ns) pts[2 * i + 1] = 0.5 * (zgrid_host[c0 + i] + zgrid_host[c0 + i + 1]);
            }
            if ((rc = enqueue_prologue(plan, pts, 2 * ns + 1, j0, nj, st))) return rc;
            double hs[kChunkSteps];
            for (int i = 0; i < ns; ++i) hs[i] = zgrid_host[c0 + i + 1] - zgrid_host[c0 + i];
            if (plan->launch == WPCCC_LAUNCH_PERSISTENT) {
                if ((rc = enqueue_chunk(plan, X, j0, nj, hs, ns, plan->stage_rows, plan->chunk_smem, st)))
                    return rc;
                continue;
            }
            if ((rc = enqueue_fpoint(plan, j0, nj, 0, st))) return rc;
            for (int i = 0; i < ns; ++i)
                if ((rc = enqueue_step(plan, X, j0, nj, 2 * i, hs[i], st))) return rc;
        }
    }
    if (P_dev || norm_dev) {
        hipError_t e = launch_probabilities((const double2*)X, plan->n_traj, plan->c.meta.n_states, plan->n_pad,
                                            (double*)P_dev, (double*)norm_dev, st, plan->timer.open(kProb));
        if ((rc = launched(e, "k_probabilities"))) return rc;
    }
    return WPCCC_OK;
}

int wpccc_adjoint(wpccc_plan_t plan, const double* zgrid_host, int n_points, const void* X0_dev, void* X_dev,
                  const void* gX_dev, void* grad_dev, void* stream) {
    clear_error();
    if (!plan || !X0_dev || !gX_dev || !grad_dev) {
        set_error("wpccc_adjoint: NULL argument");
        return WPCCC_EINVAL;
    }
    if (plan->p2c) {
        set_error("wpccc_adjoint: one-centre plans only");
        return WPCCC_ENOTSUP;
    }
    if (plan->mixed || plan->interp) {
        set_error("wpccc_adjoint: plans with the FP64 moment table only (the operator kernel reads it)");
        return WPCCC_ENOTSUP;
    }
    if (!plan->apply_ok) {
        set_error("wpccc_adjoint: basis too large for the operator kernel's LDS (%d bytes)", plan->stage_smem);
        return WPCCC_ENOTSUP;
    }
    int rc = check_grid(zgrid_host, n_points);
    if (rc) return rc;
    for (int i = 0; i < n_points; ++i)
        if (path_hits_origin(plan, zgrid_host[i]) ||
            (i + 1 < n_points && path_hits_origin(plan, 0.5 * (zgrid_host[i] + zgrid_host[i + 1])))) {
            set_error("wpccc_adjoint: R = 0 on the grid");
            return WPCCC_EINVAL;
        }
    hipStream_t st = (hipStream_t)stream;
    const int n_steps = n_points - 1;
    const size_t V = (size_t)plan->n_traj * plan->n_pad;
    // segments of K steps: the reverse sweep recomputes a segment from its
    // checkpoint keeping every state and stage input (4 K + 1 vectors), then
    // runs its steps backwards.  Default: one segment over the whole grid (no
    // checkpoints, nothing recomputed) when it takes at most kAdjointStoreAll
    // bytes, else about sqrt(n_steps) steps per segment.
    const double all_bytes = (4.0 * n_steps + 1.0) * V * sizeof(double2);
    int K = plan->ckpt_every > 0 ? plan->ckpt_every
                                 : (all_bytes <= kAdjointStoreAll ? n_steps : (int)std::ceil(std::sqrt((double)n_steps)));
    K = std::max(1, std::min(K, n_steps));
    const int n_ck = (n_steps + K - 1) / K;
    if (K > plan->adj_K || n_ck > plan->adj_nck || !plan->d_lam) {
        void* old[] = {plan->d_lam, plan->d_nu, plan->d_ckpt, plan->d_seg};
        (void)hipStreamSynchronize(st);
        for (void* q : old)
            if (q) (void)hipFree(q);
        plan->d_lam = plan->d_nu = plan->d_ckpt = plan->d_seg = nullptr;
        plan->adj_K = std::max(K, plan->adj_K);
        plan->adj_nck = std::max(n_ck, plan->adj_nck);
        long long& tot = plan->bytes;
        if ((rc = dev_alloc(&plan->d_lam, 2 * V, tot)) || (rc = dev_alloc(&plan->d_nu, 3 * V, tot)) ||
            (rc = dev_alloc(&plan->d_ckpt, (size_t)plan->adj_nck * V, tot)) ||
            (rc = dev_alloc(&plan->d_seg, (size_t)(4 * plan->adj_K + 1) * V, tot))) {
            plan->adj_K = plan->adj_nck = 0;
            return rc;
        }
        // the stage kernels write the states only: the padding entries of the
        // stored states (copied out as the final amplitudes) stay zero
        WPCCC_HIP_CHECK(hipMemsetAsync(plan->d_seg, 0, (size_t)(4 * plan->adj_K + 1) * V * sizeof(double2), st));
    }
    const size_t VB = V * sizeof(double2);
    // segment store: states x_0..x_K, then (u2, u3, u4) of each step
    double2* seg = plan->d_seg;
    auto xs_of = [&](int i) { return seg + (size_t)i * V; };
    auto us_of = [&](int i, int k) { return seg + (size_t)(K + 1 + 3 * i + k) * V; };
    AdjointPoints pts{zgrid_host, n_steps};
    // forward sweep with a checkpoint every K steps (not needed for one segment)
    if (n_ck > 1) {
        double2* xw = xs_of(0);
        WPCCC_HIP_CHECK(hipMemcpyAsync(xw, X0_dev, VB, hipMemcpyDeviceToDevice, st));
        for (int n = 0; n < n_steps; ++n) {
            if (n % K == 0)
                WPCCC_HIP_CHECK(hipMemcpyAsync(plan->d_ckpt + (size_t)(n / K) * V, xw, VB, hipMemcpyDeviceToDevice, st));
            const int pz = pts.slot(plan, n, st, &rc);
            if (rc) return rc;
            // large bases: the cached stage form, from F(pz) (the cache may hold another point)
            if (plan->gg && (rc = enqueue_fpoint(plan, 0, plan->n_traj, pz, st, 0))) return rc;
            if ((rc = enqueue_step(plan, xw, 0, plan->n_traj, pz, zgrid_host[n + 1] - zgrid_host[n], st, plan->gg)))
                return rc;
        }
        if (X_dev) WPCCC_HIP_CHECK(hipMemcpyAsync(X_dev, xw, VB, hipMemcpyDeviceToDevice, st));
    }
    // reverse sweep; lambda alternates between two buffers, nu4, nu3, nu2 are
    // the adjoint applications of stages 4, 3, 2 of the current step
    double2* lam = plan->d_lam;
    double2* lam_next = plan->d_lam + V;
    double2* nu4 = plan->d_nu;
    double2* nu3 = plan->d_nu + V;
    double2* nu2 = plan->d_nu + 2 * V;
    WPCCC_HIP_CHECK(hipMemcpyAsync(lam, gX_dev, VB, hipMemcpyDeviceToDevice, st));
    WPCCC_HIP_CHECK(hipMemsetAsync(plan->d_gpart, 0,
                                   (size_t)plan->n_traj * kGradSlots * stage_chunks(plan->c.meta, plan->apply_rows) *
                                       sizeof(double), st));
    for (int s = n_ck - 1; s >= 0; --s) {
        const int n0 = s * K, n1 = std::min(n0 + K, n_steps);
        const void* x0 = n_ck > 1 ? (const void*)(plan->d_ckpt + (size_t)s * V) : X0_dev;
        WPCCC_HIP_CHECK(hipMemcpyAsync(xs_of(0), x0, VB, hipMemcpyDeviceToDevice, st));
        for (int n = n0; n < n1; ++n) {
            const int i = n - n0;
            const int pz = pts.slot(plan, n, st, &rc);
            if (rc) return rc;
            if ((rc = stored_step(plan, pz, zgrid_host[n + 1] - zgrid_host[n], xs_of(i), xs_of(i + 1), us_of(i, 0),
                                  us_of(i, 1), us_of(i, 2), st)))
                return rc;
        }
        if (n_ck == 1 && X_dev) WPCCC_HIP_CHECK(hipMemcpyAsync(X_dev, xs_of(n1 - n0), VB, hipMemcpyDeviceToDevice, st));
        for (int n = n1 - 1; n >= n0; --n) {
            const int i = n - n0;
            const int pz = pts.slot(plan, n, st, &rc);
            if (rc) return rc;
            const double z0 = zgrid_host[n], z1 = zgrid_host[n + 1], zm = 0.5 * (z0 + z1), h = z1 - z0;
            // stage 4: mu4 = h/6 lambda
            if ((rc = enqueue_reverse_stage(plan, pz + 2, z1, lam, h / 6.0, nullptr, 0.0, nu4, {}, us_of(i, 2), st)))
                return rc;
            // stage 3: mu3 = h/3 lambda + h nu4
            if ((rc = enqueue_reverse_stage(plan, pz + 1, zm, lam, h / 3.0, nu4, h, nu3, {}, us_of(i, 1), st)))
                return rc;
            // stage 2: mu2 = h/3 lambda + h/2 nu3
            if ((rc = enqueue_reverse_stage(plan, pz + 1, zm, lam, h / 3.0, nu3, 0.5 * h, nu2, {}, us_of(i, 0), st)))
                return rc;
            // stage 1: mu1 = h/6 lambda + h/2 nu2, and
            // lambda_n = lambda_(n+1) + nu1 + nu2 + nu3 + nu4 with nu1 = M^H mu1
            if ((rc = enqueue_reverse_stage(plan, pz, z0, lam, h / 6.0, nu2, 0.5 * h, lam_next, {lam, nu2, nu3, nu4},
                                            xs_of(i), st)))
                return rc;
            std::swap(lam, lam_next);
        }
    }
    return launched(launch_grad_sum(plan->d_gpart, stage_chunks(plan->c.meta, plan->apply_rows), (double*)grad_dev,
                                    plan->n_traj, st),
                    "k_grad_sum");
}

int wpccc_plan_timing(wpccc_plan_t plan, int enable) {
    if (!plan) {
        set_error("wpccc_plan_timing: NULL plan");
        return WPCCC_EINVAL;
    }
    if (!enable) {
        WPCCC_HIP_CHECK(hipDeviceSynchronize());
        plan->timer.recycle_all();
    }
    plan->timer.on = enable != 0;
    return WPCCC_OK;
}

int wpccc_plan_kernel_time(wpccc_plan_t plan, const char* kernel, double* total_ms, long long* launches) {
    if (!plan || !kernel) {
        set_error("wpccc_plan_kernel_time: NULL argument");
        return WPCCC_EINVAL;
    }
    int id = -1;
    for (int k = 0; k < kNumKernels; ++k)
        if (std::strcmp(kernel, kKernelNames[k]) == 0) id = k;
    if (id < 0) {
        set_error("wpccc_plan_kernel_time: unknown kernel '%s'", kernel);
        return WPCCC_EINVAL;
    }
    return plan->timer.take(id, total_ms, launches);
}

int wpccc_plan_groups(wpccc_plan_t plan, int* n_groups, int* group_of_traj_host) {
    if (!plan) {
        set_error("wpccc_plan_groups: NULL plan");
        return WPCCC_EINVAL;
    }
    if (n_groups) *n_groups = plan->obs.n_groups;
    if (group_of_traj_host)
        std::memcpy(group_of_traj_host, plan->obs.group_of.data(), plan->obs.group_of.size() * sizeof(int));
    return WPCCC_OK;
}

int wpccc_observables(wpccc_plan_t plan, const void* P_dev, void* chan_dev, void* sigma_dev, void* stream) {
    clear_error();
    if (!plan || !P_dev || !chan_dev) {
        set_error("wpccc_observables: NULL plan, P_dev or chan_dev");
        return WPCCC_EINVAL;
    }
    const hipError_t e = launch_observables(plan->obs, (const double*)P_dev, (double*)chan_dev, (double*)sigma_dev,
                                            (hipStream_t)stream, plan->timer.open(kChannels));
    return launched(e, "k_channels");
}

}  // extern "C"

namespace wpccc {

const char* const kKernelNames[kNumKernels] = {
    "k_stage",        "k_slot_setup",  "k_couplings_dense", "k_probabilities", "k_moments",    "k_prologue",
    "k_2c_nodes",     "k_2c_interp",   "k_2c_contract", "k_2c_assemble",     "k_setup_batch",   "k_2c_direct",  "k_lu_panel",
    "k_lu_swap_trsm", "k_lu_update",   "k_2c_hu",           "k_2c_solve",      "k_2c_finish",  "k_chunk",
    "k_2c_reduce",    "k_fpoint",      "k_channels",    "k_lu_check",        "k_lu_rhs",
    "k_2c_dk",        "k_2c_symm"};

LaunchEv KernelTimer::open(int kernel) {
    LaunchEv ev;
    if (!on) return ev;
    Rec r{kernel, nullptr, nullptr};
    for (hipEvent_t* e : {&r.a, &r.b}) {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            *e = nullptr;
        }
    }
    if (!r.a || !r.b) {
        if (r.a) pool.push_back(r.a);
        if (r.b) pool.push_back(r.b);
        return ev;
    }
    recs.push_back(r);
    ev.a = r.a;
    ev.b = r.b;
    return ev;
}

void KernelTimer::recycle_all() {
    for (auto& r : recs) {
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
}

int KernelTimer::take(int kernel, double* total_ms, long long* launches) {
    double tot = 0.0;
    long long n = 0;
    std::vector<Rec> keep;
    for (auto& r : recs) {
        if (r.kernel != kernel) {
            keep.push_back(r);
            continue;
        }
        WPCCC_HIP_CHECK(hipEventSynchronize(r.b));
        float ms = 0.f;
        // a launcher that had nothing to do records neither event: not a launch
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            tot += ms;
            ++n;
        } else {
            (void)hipGetLastError();
        }
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.swap(keep);
    if (total_ms) *total_ms = tot;
    if (launches) *launches = n;
    return WPCCC_OK;
}

KernelTimer::~KernelTimer() {
    recycle_all();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace wpccc

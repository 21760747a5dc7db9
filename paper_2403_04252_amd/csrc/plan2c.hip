// Two-centre plan (Eq. 1 with electron capture): host side.
//
// Paths are grouped by their (target, projectile) basis pair; each group
// holds both centres' Eq. D1 tables, its Meta2C and, per path, three coupling
// slots (z, z_mid, z_new of Algorithm 1) with S, its LU factors and H.  A
// step computes the couplings of the positions not yet held (normally z_mid
// and z_new, z being the previous step's z_new), factorises S at each and
// runs the four RK4 stages.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "plan2c.h"

namespace wpccc {

namespace {

// ---------------------------------------------------------------------------
// Quadrature nodes (host, once per plan)
// ---------------------------------------------------------------------------

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal d and off-diagonal e (e[0] unused), by the Sturm sequence of its
// leading minors.
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
    int cnt = 0;
    double q = 1.0;
    for (size_t k = 0; k < d.size(); ++k) {
        const double off = k ? e[k] * e[k] / q : 0.0;
        q = d[k] - x - off;
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Gauss-Laguerre nodes x_i of L_n (ascending) and the scaled weights
// w_i e^{x_i}.  The nodes are the eigenvalues of the Jacobi matrix of the
// Laguerre polynomials (diagonal 2k+1, off-diagonal k), isolated by
// bisection on Sturm counts and polished by Newton steps on L_n; the weights
// follow from w_i = x_i / ((n+1)^2 L_{n+1}(x_i)^2), evaluated with the
// recurrence for e^{-x/2} L_k(x), which stays bounded for large x.
void gauss_laguerre_scaled(int n, std::vector<double>& x, std::vector<double>& ws) {
    std::vector<double> d(n), e(n, 0.0);
    for (int k = 0; k < n; ++k) d[k] = 2.0 * k + 1.0;
    for (int k = 1; k < n; ++k) e[k] = k;
    x.assign(n, 0.0);
    ws.assign(n, 0.0);
    const double hi = 4.0 * n + 2.0;
    for (int i = 0; i < n; ++i) {
        double lo = 0.0, up = hi;
        for (int it = 0; it < 200 && up - lo > 1e-15 * std::max(1.0, up); ++it) {
            const double mid = 0.5 * (lo + up);
            if (sturm_count(d, e, mid) > i) up = mid;
            else lo = mid;
        }
        double xi = 0.5 * (lo + up);
        for (int it = 0; it < 3; ++it) {
            double p0 = std::exp(-xi / 2.0), p1 = (1.0 - xi) * p0;  // scaled L_0, L_1
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0 - xi) * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            // L_n' = n (L_n - L_{n-1}) / x; the scale factor cancels in the ratio
            const double den = n * (p1 - p0);
            if (den != 0.0) xi -= xi * p1 / den;
        }
        double p0 = std::exp(-xi / 2.0), p1 = (1.0 - xi) * p0;
        for (int k = 1; k <= n; ++k) {
            const double p2 = ((2.0 * k + 1.0 - xi) * p1 - k * p0) / (k + 1.0);
            p0 = p1;
            p1 = p2;
        }
        x[i] = xi;
        ws[i] = xi / ((n + 1.0) * (n + 1.0) * p1 * p1);
    }
}

// Gauss-Legendre nodes (ascending) and weights: Newton on P_n from the
// cosine estimates of its zeros, w = 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double t = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = t;
            for (int k = 1; k < n; ++k) {
                const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        x[n - 1 - i] = t;
        w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------

struct Group2C {
    const HostBasis* tb = nullptr;
    const HostBasis* pb = nullptr;
    Centre cT, cP;
    Meta2C m{};
    Meta2C* d_m = nullptr;
    std::vector<int> paths;  // global path of each local path
    int* d_paths = nullptr;
    std::vector<int2> tiles;
    int2* d_tiles = nullptr;
    double *d_phiT_T = nullptr, *d_phiT_P = nullptr;
    int *d_radl_T = nullptr, *d_radl_P = nullptr;
    double2 *d_S = nullptr, *d_LU = nullptr, *d_H = nullptr;  // [path][slot][N*N]
    double2* d_M = nullptr;  // [path][slot][N*N] S^{-1} H (explicit form only)
    double2* d_dK = nullptr; // [path][2][NT*NP] dK/dz (symmetric form only)
    int* d_piv = nullptr;                                      // [path][slot][N]
    int* d_perm = nullptr;                                     // [path][slot][N]
    int* d_skip = nullptr;                                     // [path][slot] no-pivot block form (k_lu_check)
    int max_jobs = 0;
    double* d_nodes = nullptr;
    int* d_jst = nullptr;
    int* d_nact = nullptr;
    double* d_tmol = nullptr;
    int2 *d_rinfoT = nullptr, *d_rinfoP = nullptr;
    void *d_AT = nullptr, *d_BT = nullptr;  // interpolated operands [job][rows][n_nodes]
    double *d_FrowT = nullptr, *d_GT = nullptr, *d_FrowP = nullptr, *d_GP = nullptr;
    double2 *d_PHT = nullptr, *d_PHP = nullptr;
};

struct Plan2C {
    std::vector<Group2C> groups;
    std::vector<int> group_of, local_of;
    int n_traj = 0, n_pad = 0, batched = 1, q_prior = 0, n_eta = 0, n_tau = 0, mixed = 0;
    int explicit_m = 0;  // M = S^{-1} H formed per coupling point (WPCCC_SOLVE_EXPLICIT)
    // stage kernels: one launch over every group's paths (batched 1) or per group (batched 2)
    bool stage_all = true;
    PathMats* d_pm = nullptr;       // [n_traj] ordered by group, then local path
    std::vector<int> pm_first;      // first entry of each group in d_pm
    int N_max = 0;
    int symmetric = 0;   // S-norm-conserving form of H (opts.symmetric)
    double dz_sym = 1e-4;
    std::vector<double> b, v;
    double *d_b = nullptr, *d_v = nullptr;
    int* d_flag = nullptr;  // [0] non-finite amplitude, [1] singular path + 1, [2] its pivot row
    double2 *d_Ua = nullptr, *d_Ub = nullptr, *d_Xacc = nullptr, *d_Y = nullptr;
    double *d_xlag = nullptr, *d_wlag = nullptr, *d_tleg = nullptr, *d_wleg = nullptr;
    long long bytes = 0;
    KernelTimer* timer = nullptr;
    // one stream per group (groups are independent within a step): the
    // latency-bound LU panels and solves of one group overlap the contraction
    // of another; fork and join on the caller's stream every step
    std::vector<hipStream_t> gstreams;
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;
    double slot_z[kSlots2C];
    bool slot_ok[kSlots2C] = {};
    // graph replay of wpccc_propagate's steps (opts.graph): a step whose start
    // point is already held replays the graph captured for that slot (the
    // slots of z_mid and z_new follow from it); the step's z_mid, z_new and h
    // come from d_zh[3 * *d_step + k], and the graph's last node advances
    // *d_step.  A graph bakes in X and d_zh: either changing captures again.
    bool use_graph = false, capturing = false;
    hipGraphExec_t gexec[kSlots2C] = {};
    // pipelined replays (one launch over every group's stages): graph step i
    // runs the stages of step i and forms the couplings of step i + 1 on the
    // group streams (zahead = 1 while such a graph is captured); one graph
    // per slot assignment (pexec, keyed by pipe_key)
    int zahead = 0;
    std::vector<std::pair<int, hipGraphExec_t>> pexec;
    hipStream_t pstream = nullptr;      // coupling stream of a one-group plan
    hipEvent_t pfork = nullptr;
    std::vector<hipEvent_t> pjoin;
    double2* gX = nullptr;
    hipStream_t gcap = nullptr;
    double* d_zh = nullptr;
    double* h_zh = nullptr;   // pinned staging of d_zh
    int zh_cap = 0;           // steps d_zh holds
    int* d_step = nullptr;
    hipEvent_t zh_copied = nullptr;
};

namespace {

// launch with optional event timing
template <typename F>
int timed(Plan2C* p, int id, F&& launch) {
    return launched(launch(p->timer->open(id)), kKernelNames[id]);
}

void free_group(Group2C& g) {
    centre_free(g.cT);
    centre_free(g.cP);
    void* bufs[] = {g.d_m,    g.d_paths, g.d_tiles, g.d_phiT_T, g.d_phiT_P, g.d_radl_T, g.d_radl_P,
                    g.d_S,    g.d_LU,    g.d_H,     g.d_piv,    g.d_perm,   g.d_skip,   g.d_nodes,  g.d_jst,    g.d_nact,
                    g.d_tmol, g.d_FrowT, g.d_GT,    g.d_FrowP,  g.d_GP,     g.d_PHT,    g.d_PHP,
                    g.d_rinfoT, g.d_rinfoP, g.d_AT, g.d_BT, g.d_M, g.d_dK};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
}

int check_basis(const HostBasis& hb, const char* who) {
    if (hb.spec.l_max > kMaxL) {
        set_error("wpccc_plan_create_2c: %s basis l_max %d exceeds %d", who, hb.spec.l_max, kMaxL);
        return WPCCC_EINVAL;
    }
    if (hb.n_r < 4) {
        set_error("wpccc_plan_create_2c: %s basis needs at least 4 grid intervals", who);
        return WPCCC_EINVAL;
    }
    return WPCCC_OK;
}

// Meta2C of one basis pair.
void fill_meta(const HostBasis& tb, const HostBasis& pb, int n_eta, int n_tau, int q_prior, int same, int mixed,
               Meta2C& m, std::vector<int2>& tiles) {
    std::memset(&m, 0, sizeof m);
    m.LT = tb.spec.l_max;
    m.LP = pb.spec.l_max;
    m.L = std::max(m.LT, m.LP);
    m.NT = tb.n_states;
    m.NP = pb.n_states;
    m.N = m.NT + m.NP;
    m.nfT = tb.n_f;
    m.nfP = pb.n_f;
    m.nrT = tb.n_r;
    m.nrP = pb.n_r;
    m.rmaxT = tb.spec.r_max;
    m.rmaxP = pb.spec.r_max;
    m.ZT = tb.spec.Z;
    m.ZP = pb.spec.Z;
    m.n_eta = n_eta;
    m.n_tau = n_tau;
    m.n_nodes = n_eta * n_tau;
    m.f_pa = kFJ + 2 * m.L + 1;
    m.f_pb = m.f_pa + (m.LT + 1) * (m.LT + 2) / 2;
    m.n_fields = m.f_pb + (m.LP + 1) * (m.LP + 2) / 2;
    m.same = same;
    m.mirror = q_prior && same;
    m.n_w = (q_prior && !m.mirror) ? 3 : 2;
    m.q_prior = q_prior;
    m.mixed = mixed;
    for (int l = 0; l <= kMaxL + 1; ++l) {
        m.radT_off[l] = l <= m.LT ? tb.rad_off[l] : tb.n_f;
        m.radP_off[l] = l <= m.LP ? pb.rad_off[l] : pb.n_f;
        m.stT_off[l] = l <= m.LT ? tb.state_off[l] : tb.n_states;
        m.stP_off[l] = l <= m.LP ? pb.state_off[l] : pb.n_states;
    }
    for (int l = 0; l <= kMaxL; ++l) {
        m.nA[l] = l <= m.LT ? tb.n_f - tb.rad_off[l] : 0;
        m.nB[l] = l <= m.LP ? pb.n_f - pb.rad_off[l] : 0;
        m.n_lT[l] = l <= m.LT ? tb.n_l[l] : 0;
        m.n_lP[l] = l <= m.LP ? pb.n_l[l] : 0;
    }
    tiles.clear();
    int off = 0;
    for (int s = 0; s <= m.LT; ++s)
        for (int t = 0; t <= m.LP; ++t) {
            m.st_off[s][t] = off;
            const int nw = st_nw(m.same, m.n_w, s, t);
            if (!nw) continue;   // formed from block (t, s)
            off += st_nk(s, t, nw) * m.nA[s] * m.nB[t];
            for (int a0 = 0; a0 < m.nA[s]; a0 += kTile)
                for (int b0 = 0; b0 < m.nB[t]; b0 += kTile)
                    tiles.push_back(make_int2(s | (t << 8) | (overlap_mirrored(m.same, s, t, a0, b0) ? kTileUpper : 0),
                                              a0 | (b0 << 16)));
        }
    // heaviest tiles first (weights formed x active 16 x 16 subtiles): the
    // dispatcher takes each XCD's work items in order, so the last ones it
    // hands out are the short ones; the order changes no sum
    auto tile_cost = [&](const int2& q) {
        const int s = q.x & 0xff, t = (q.x >> 8) & 0xff, a0 = q.y & 0xffff, b0 = q.y >> 16;
        const int nk = (q.x & kTileUpper) ? st_nk(s, t, 1) : st_nk(s, t, st_nw(m.same, m.n_w, s, t));
        return nk * (a0 + 16 < m.nA[s] ? 2 : 1) * (b0 + 16 < m.nB[t] ? 2 : 1);
    };
    std::stable_sort(tiles.begin(), tiles.end(),
                     [&](const int2& x, const int2& y) { return tile_cost(x) > tile_cost(y); });
    m.n_tmol = off;
    m.n_tiles = (int)tiles.size();
    m.n_split = kContractSplit;
    m.rowsT = m.rowsP = 0;
    for (int l = 0; l <= kMaxL; ++l) {
        m.rowT_off[l] = m.rowsT;
        m.rowP_off[l] = m.rowsP;
        m.rowsT += m.nA[l];
        m.rowsP += m.nB[l];
    }
}

std::vector<double> transposed_phi(const HostBasis& hb) {
    std::vector<double> t((size_t)(hb.n_r + 1) * hb.n_f);
    for (int a = 0; a < hb.n_f; ++a)
        for (int i = 0; i <= hb.n_r; ++i) t[(size_t)i * hb.n_f + a] = hb.phi[(size_t)a * (hb.n_r + 1) + i];
    return t;
}

std::vector<int> radial_l(const HostBasis& hb) {
    std::vector<int> r(hb.n_f, 0);
    for (int l = 0; l <= hb.spec.l_max; ++l)
        for (int n = 0; n < hb.n_l[l]; ++n) r[hb.rad_off[l] + n] = l;
    return r;
}

int upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (!bytes) return WPCCC_OK;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        set_error("host to device copy failed: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

int build_group(Plan2C* p, Group2C& g, hipStream_t st) {
    int rc;
    if ((rc = centre_build(*g.tb, st, g.cT))) return rc;
    if ((rc = centre_build(*g.pb, st, g.cP))) return rc;
    // one basis object on both centres: the overlap of the blocks s > t and
    // the prior block follow by the tau -> -tau symmetry of the quadrature
    // (k_2c_assemble)
    fill_meta(*g.tb, *g.pb, p->n_eta, p->n_tau, p->q_prior, g.tb == g.pb, p->mixed, g.m, g.tiles);
    long long& tot = p->bytes;
    tot += g.cT.bytes + g.cP.bytes;
    const Meta2C& m = g.m;
    const size_t np = g.paths.size();
    const size_t NN = (size_t)m.N * m.N;
    g.max_jobs = 2 * (p->batched ? (int)np : 1);
    const size_t J = (size_t)g.max_jobs;
    const std::vector<double> phT = transposed_phi(*g.tb), phP = transposed_phi(*g.pb);
    const std::vector<int> rlT = radial_l(*g.tb), rlP = radial_l(*g.pb);
    // operand rows: (radial index, node field of its Legendre factor) per (s, i)
    std::vector<int2> riT, riP;
    for (int s = 0; s <= m.LT; ++s)
        for (int i = 0; i < m.nA[s]; ++i) {
            const int a = m.radT_off[s] + i, l = rlT[a];
            riT.push_back(make_int2(a, m.f_pa + l * (l + 1) / 2 + s));
        }
    for (int t = 0; t <= m.LP; ++t)
        for (int i = 0; i < m.nB[t]; ++i) {
            const int b = m.radP_off[t] + i, l = rlP[b];
            riP.push_back(make_int2(b, m.f_pb + l * (l + 1) / 2 + t));
        }
    const size_t esz = p->mixed ? sizeof(float) : sizeof(double);
    if ((rc = dev_alloc(&g.d_m, 1, tot))) return rc;
    if ((rc = dev_alloc(&g.d_paths, np, tot))) return rc;
    if ((rc = dev_alloc(&g.d_tiles, g.tiles.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_phiT_T, phT.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_phiT_P, phP.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_radl_T, rlT.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_radl_P, rlP.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_S, np * kSlots2C * NN, tot))) return rc;
    if ((rc = dev_alloc(&g.d_LU, np * kSlots2C * NN, tot))) return rc;
    if ((rc = dev_alloc(&g.d_H, np * kSlots2C * NN, tot))) return rc;
    if (p->explicit_m && (rc = dev_alloc(&g.d_M, np * kSlots2C * NN, tot))) return rc;
    if (p->symmetric && (rc = dev_alloc(&g.d_dK, np * 2 * (size_t)m.NT * m.NP, tot))) return rc;
    if ((rc = dev_alloc(&g.d_piv, np * kSlots2C * m.N, tot))) return rc;
    if ((rc = dev_alloc(&g.d_perm, np * kSlots2C * m.N, tot))) return rc;
    if ((rc = dev_alloc(&g.d_skip, np * kSlots2C, tot))) return rc;
    if ((rc = dev_alloc(&g.d_nodes, J * m.n_fields * m.n_nodes, tot))) return rc;
    if ((rc = dev_alloc(&g.d_jst, J * 2 * m.n_nodes, tot))) return rc;
    if ((rc = dev_alloc(&g.d_nact, J, tot))) return rc;
    if ((rc = dev_alloc(&g.d_tmol, J * (size_t)m.n_split * m.n_tmol, tot))) return rc;
    if ((rc = dev_alloc(&g.d_rinfoT, riT.size(), tot))) return rc;
    if ((rc = dev_alloc(&g.d_rinfoP, riP.size(), tot))) return rc;
    if ((rc = dev_alloc_bytes(&g.d_AT, J * m.rowsT * (size_t)m.n_nodes * esz, tot))) return rc;
    if ((rc = dev_alloc_bytes(&g.d_BT, J * m.rowsP * (size_t)m.n_nodes * esz, tot))) return rc;
    if ((rc = dev_alloc(&g.d_FrowT, J * g.cT.meta.n_frow, tot))) return rc;
    if ((rc = dev_alloc(&g.d_GT, J * g.cT.meta.n_g, tot))) return rc;
    if ((rc = dev_alloc(&g.d_PHT, J * m.NT, tot))) return rc;
    if ((rc = dev_alloc(&g.d_FrowP, J * g.cP.meta.n_frow, tot))) return rc;
    if ((rc = dev_alloc(&g.d_GP, J * g.cP.meta.n_g, tot))) return rc;
    if ((rc = dev_alloc(&g.d_PHP, J * m.NP, tot))) return rc;
    if ((rc = upload(g.d_m, &g.m, sizeof(Meta2C), st))) return rc;
    if ((rc = upload(g.d_paths, g.paths.data(), np * sizeof(int), st))) return rc;
    if ((rc = upload(g.d_tiles, g.tiles.data(), g.tiles.size() * sizeof(int2), st))) return rc;
    if ((rc = upload(g.d_phiT_T, phT.data(), phT.size() * sizeof(double), st))) return rc;
    if ((rc = upload(g.d_phiT_P, phP.data(), phP.size() * sizeof(double), st))) return rc;
    if ((rc = upload(g.d_radl_T, rlT.data(), rlT.size() * sizeof(int), st))) return rc;
    if ((rc = upload(g.d_radl_P, rlP.data(), rlP.size() * sizeof(int), st))) return rc;
    if ((rc = upload(g.d_rinfoT, riT.data(), riT.size() * sizeof(int2), st))) return rc;
    if ((rc = upload(g.d_rinfoP, riP.data(), riP.size() * sizeof(int2), st))) return rc;
    // the host vectors above are released on return: wait for the copies
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    return WPCCC_OK;
}

// Couplings of local paths [l0, l0 + np) of group g at n_sub positions
// (slot[k], z[k]): D_T and D_P, K and Q (and the prior block), then LU of S.
int enqueue_rhs(Plan2C* p, Group2C& g, int l0, int np, int n_sub, const int* slot, hipStream_t st);

// factor: also the LU of S (and, in the explicit form outside the symmetric
// one, M = S^{-1} H); false for the positions that only feed dS/dz
int enqueue_couplings(Plan2C* p, Group2C& g, int l0, int np, int n_sub, const int* slot, const double* z,
                      hipStream_t st, bool factor = true) {
    Jobs J{};
    J.path0 = l0;
    J.n_sub = n_sub;
    for (int k = 0; k < n_sub; ++k) {
        J.slot[k] = slot[k];
        J.z[k] = z[k];
    }
    if (p->capturing && n_sub == 2) {
        J.zdev = p->d_zh;
        J.step = p->d_step;
        J.ahead = p->zahead;
    }
    const int nj = np * n_sub;
    int rc;
    for (int side = 0; side < 2; ++side) {
        const Centre& c = side ? g.cP : g.cT;
        SetupBatchArgs a;
        a.meta = c.d_meta;
        a.tb = c.tables(p->d_b, p->d_v);
        a.jobs = J;
        a.paths = g.d_paths;
        a.parity = side ? -1 : 1;
        a.Frow = side ? g.d_FrowP : g.d_FrowT;
        a.G = side ? g.d_GP : g.d_GT;
        a.PH = side ? g.d_PHP : g.d_PHT;
        a.nbF = (c.meta.n_frow + 255) / 256;
        a.nbP = (c.meta.n_states + 255) / 256;
        if ((rc = timed(p, k2cSetup, [&](const LaunchEv& ev) { return launch_setup_batch(a, c.meta, nj, st, ev); }))) return rc;
    }
    {
        DirectArgs a;
        a.mT = g.cT.d_meta;
        a.mP = g.cP.d_meta;
        a.m = g.d_m;
        a.jobs = J;
        a.FrowT = g.d_FrowT;
        a.GT = g.d_GT;
        a.PHT = g.d_PHT;
        a.FrowP = g.d_FrowP;
        a.GP = g.d_GP;
        a.PHP = g.d_PHP;
        a.n_frowT = g.cT.meta.n_frow;
        a.n_gT = g.cT.meta.n_g;
        a.n_frowP = g.cP.meta.n_frow;
        a.n_gP = g.cP.meta.n_g;
        a.H = g.d_H;
        if ((rc = timed(p, k2cDirect, [&](const LaunchEv& ev) { return launch_2c_direct(a, g.m, nj, st, ev); }))) return rc;
    }
    {
        NodeArgs a;
        a.m = g.d_m;
        a.jobs = J;
        a.xlag = p->d_xlag;
        a.wlag = p->d_wlag;
        a.tleg = p->d_tleg;
        a.wleg = p->d_wleg;
        a.paths = g.d_paths;
        a.bvec = p->d_b;
        a.vvec = p->d_v;
        a.nodes = g.d_nodes;
        a.jst = g.d_jst;
        a.n_act = g.d_nact;
        if ((rc = timed(p, k2cNodes, [&](const LaunchEv& ev) { return launch_2c_nodes(a, g.m, nj, st, ev); }))) return rc;
    }
    {
        InterpArgs ia;
        ia.m = g.d_m;
        ia.phiT_T = g.d_phiT_T;
        ia.phiT_P = g.d_phiT_P;
        ia.rinfoT = g.d_rinfoT;
        ia.rinfoP = g.d_rinfoP;
        ia.nodes = g.d_nodes;
        ia.jst = g.d_jst;
        ia.n_act = g.d_nact;
        ia.AT = g.d_AT;
        ia.BT = g.d_BT;
        if ((rc = timed(p, k2cInterp, [&](const LaunchEv& ev) { return launch_2c_interp(ia, g.m, nj, st, ev); })))
            return rc;
        ContractArgs a;
        a.m = g.d_m;
        a.n_jobs = nj;
        a.tiles = g.d_tiles;
        a.AT = g.d_AT;
        a.BT = g.d_BT;
        a.nodes = g.d_nodes;
        a.n_act = g.d_nact;
        a.tmol = g.d_tmol;
        if ((rc = timed(p, k2cContract, [&](const LaunchEv& ev) { return launch_2c_contract(a, g.m, nj, st, ev); }))) return rc;
        if ((rc = timed(p, k2cReduce, [&](const LaunchEv& ev) { return launch_2c_reduce(g.d_tmol, g.m, nj, st, ev); })))
            return rc;
    }
    {
        AssembleArgs a;
        a.m = g.d_m;
        a.jobs = J;
        a.paths = g.d_paths;
        a.bvec = p->d_b;
        a.vvec = p->d_v;
        a.epsT = g.cT.d_eps;
        a.epsP = g.cP.d_eps;
        a.tmol = g.d_tmol;
        a.S = g.d_S;
        a.LU = g.d_LU;
        a.H = g.d_H;
        if ((rc = timed(p, k2cAssemble, [&](const LaunchEv& ev) { return launch_2c_assemble(a, g.m, nj, st, ev); }))) return rc;
    }
    if (!factor) return WPCCC_OK;
    // LU of S with partial pivoting: the first N_T columns by the no-pivot
    // block form where k_lu_check allows it (see LUStepArgs), else by panels
    LUStepArgs a{};
    a.N = g.m.N;
    a.jobs = J;
    a.LU = g.d_LU;
    a.piv = g.d_piv;
    a.perm = g.d_perm;
    a.paths = g.d_paths;
    a.flag = p->d_flag;
    a.skip = g.d_skip;
    a.nt = g.m.NT;
    if ((rc = timed(p, kLuCheck, [&](const LaunchEv& ev) { return launch_lu_check(a, nj, st, ev); }))) return rc;
    a.k0 = 0;
    a.nb = g.m.NT;
    a.skip_mode = 2;
    if ((rc = timed(p, kLuUpdate, [&](const LaunchEv& ev) { return launch_lu_update(a, nj, st, ev); }))) return rc;
    const int pw = lu_panel_width(g.m.N);
    auto panels = [&](int from, int to) -> int {
        for (int k0 = from; k0 < to; k0 += pw) {
            a.k0 = k0;
            a.nb = std::min(pw, to - k0);
            int r;
            if ((r = timed(p, kLuPanel, [&](const LaunchEv& ev) { return launch_lu_panel(a, nj, st, ev); }))) return r;
            if ((r = timed(p, kLuSwap, [&](const LaunchEv& ev) { return launch_lu_swap_trsm(a, nj, st, ev); }))) return r;
            if ((r = timed(p, kLuUpdate, [&](const LaunchEv& ev) { return launch_lu_update(a, nj, st, ev); }))) return r;
        }
        return WPCCC_OK;
    };
    a.skip_mode = 1;
    if ((rc = panels(0, g.m.NT))) return rc;
    a.skip_mode = 0;
    if ((rc = panels(g.m.NT, g.m.N))) return rc;
    // the symmetric form replaces H first (enqueue_symm) and forms M after it
    return p->symmetric ? WPCCC_OK : enqueue_rhs(p, g, l0, np, n_sub, slot, st);
}

// M = S^{-1} H at the given slots (explicit form; nothing otherwise)
int enqueue_rhs(Plan2C* p, Group2C& g, int l0, int np, int n_sub, const int* slot, hipStream_t st) {
    if (!p->explicit_m) return WPCCC_OK;
    RhsArgs ra{};
    ra.N = g.m.N;
    ra.jobs.path0 = l0;
    ra.jobs.n_sub = n_sub;
    for (int k = 0; k < n_sub; ++k) ra.jobs.slot[k] = slot[k];
    ra.LU = g.d_LU;
    ra.perm = g.d_perm;
    ra.H = g.d_H;
    ra.M = g.d_M;
    return timed(p, kLuRhs, [&](const LaunchEv& ev) { return launch_lu_rhs(ra, np * n_sub, st, ev); });
}

SymArgs sym_args(const Plan2C* p, Group2C& g, int l0) {
    SymArgs a{};
    a.N = g.m.N;
    a.NT = g.m.NT;
    a.NP = g.m.NP;
    a.path0 = l0;
    a.paths = g.d_paths;
    a.vvec = p->d_v;
    a.S = g.d_S;
    a.H = g.d_H;
    a.dK = g.d_dK;
    a.inv_2dz = 0.5 / p->dz_sym;
    return a;
}

// dK/dz at zp into dK buffer `which`: S at zp + dz and zp - dz computed into
// slots sa and sb (whose contents are given up)
int enqueue_dk(Plan2C* p, Group2C& g, int l0, int np, double zp, int sa, int sb, int which, hipStream_t st) {
    const int sl[2] = {sa, sb};
    const double zz[2] = {zp + p->dz_sym, zp - p->dz_sym};
    int rc;
    if ((rc = enqueue_couplings(p, g, l0, np, 2, sl, zz, st, false))) return rc;
    SymArgs a = sym_args(p, g, l0);
    a.slot_p = sa;
    a.slot_m = sb;
    a.which = which;
    return timed(p, k2cDk, [&](const LaunchEv& ev) { return launch_2c_dk(a, np, st, ev); });
}

// H at slot <- its S-norm-conserving form with dK buffer `which`
int enqueue_symm(Plan2C* p, Group2C& g, int l0, int np, int slot, int which, hipStream_t st) {
    SymArgs a = sym_args(p, g, l0);
    a.slot = slot;
    a.which = which;
    return timed(p, k2cSymm, [&](const LaunchEv& ev) { return launch_2c_symm(a, np, st, ev); });
}

// One RK4 stage for the np paths of pm (entries of d_pm), N <= N_max.
int enqueue_stage(Plan2C* p, const PathMats* pm, int np, int N_max, int stage, int slot, double h,
                  const double2* u_in, double2* X, double2* u_out, hipStream_t st) {
    Stage2CArgs a{};
    a.N_max = N_max;
    a.n_pad = p->n_pad;
    a.stage = stage;
    a.h = h;
    a.slot = slot;
    a.pm = pm;
    a.vvec = p->d_v;
    a.solve = !p->explicit_m;
    a.u_in = u_in;
    a.Y = p->d_Y;
    a.X = X;
    a.Xacc = p->d_Xacc;
    a.u_out = u_out;
    a.flag = p->d_flag;
    if (p->capturing) {
        a.hdev = p->d_zh;
        a.step = p->d_step;
    }
    int rc = timed(p, k2cHu, [&](const LaunchEv& ev) { return launch_2c_hu(a, np, st, ev); });
    if (rc) return rc;
    return timed(p, k2cSolve, [&](const LaunchEv& ev) { return launch_2c_solve(a, np, st, ev); });
}

int find_slot(const Plan2C* p, double z) {
    for (int s = 0; s < kSlots2C; ++s)
        if (p->slot_ok[s] && p->slot_z[s] == z) return s;
    return -1;
}

bool hits_origin(const Plan2C* p, double z) {
    for (double b : p->b)
        if (!(std::sqrt(b * b + z * z) > 0.0)) return true;
    return false;
}

// Coupling slots of one step z -> z + h: s0 holds z (have0: the couplings
// there are already computed), sm and sn receive z + h/2 and z + h.
struct StepSlots {
    bool have0;
    int s0, sm, sn;
};

StepSlots slots_with_start(int s0, bool have0) {
    StepSlots s{have0, s0, -1, -1};
    for (int k = 0; k < kSlots2C && s.sn < 0; ++k) {
        if (k == s0) continue;
        if (s.sm < 0) s.sm = k;
        else s.sn = k;
    }
    return s;
}

StepSlots step_slots(const Plan2C* p, double z) {
    const int s0 = find_slot(p, z);
    return s0 >= 0 ? slots_with_start(s0, true) : slots_with_start(0, false);
}

// every path keeps its own slots, so they hold these positions for all paths
void commit_slots(Plan2C* p, const StepSlots& s, double z, double h) {
    for (int k = 0; k < kSlots2C; ++k) p->slot_ok[k] = false;
    p->slot_ok[s.s0] = p->slot_ok[s.sm] = p->slot_ok[s.sn] = true;
    p->slot_z[s.s0] = z;
    p->slot_z[s.sm] = z + 0.5 * h;
    p->slot_z[s.sn] = z + h;
}

// The RK4 stages from `first` (1, or 2 when stage 1 ran already) of a step
// for the np paths of pm.
int enqueue_stages(Plan2C* p, const PathMats* pm, int np, int N_max, const StepSlots& ss, double h, double2* X,
                   hipStream_t st, int first = 1) {
    int rc;
    if (first <= 1 && (rc = enqueue_stage(p, pm, np, N_max, 1, ss.s0, h, X, X, p->d_Ua, st))) return rc;
    if ((rc = enqueue_stage(p, pm, np, N_max, 2, ss.sm, h, p->d_Ua, X, p->d_Ub, st))) return rc;
    if ((rc = enqueue_stage(p, pm, np, N_max, 3, ss.sm, h, p->d_Ub, X, p->d_Ua, st))) return rc;
    return enqueue_stage(p, pm, np, N_max, 4, ss.sn, h, p->d_Ua, X, nullptr, st);
}

// The launches of one RK4 step of every path in the given slots.
int enqueue_step_slots(Plan2C* p, double2* X, double z, double h, const StepSlots& ss, hipStream_t st,
                       bool with_stages = true) {
    const double zm = z + 0.5 * h, zn = z + h;
    int rc;
    const bool fork = !p->gstreams.empty();
    if (fork) WPCCC_HIP_CHECK(hipEventRecord(p->fork_ev, st));
    // stage 1 reads the couplings at z only: where they are held it runs on
    // st while the group streams form those at z + h/2 and z + h (it touches
    // none of their slots, and they none of its vectors)
    const bool early1 = with_stages && p->stage_all && ss.have0 && fork;
    if (early1 && (rc = enqueue_stage(p, p->d_pm, p->n_traj, p->N_max, 1, ss.s0, h, X, X, p->d_Ua, st))) return rc;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        Group2C& g = p->groups[gi];
        hipStream_t gs = st;
        if (fork) {
            gs = p->gstreams[gi];
            WPCCC_HIP_CHECK(hipStreamWaitEvent(gs, p->fork_ev, 0));
        }
        const int npath = (int)g.paths.size();
        const int chunk = p->batched ? npath : 1;
        for (int l0 = 0; l0 < npath; l0 += chunk) {
            const int np = std::min(chunk, npath - l0);
            if (!ss.have0) {
                const int sl[1] = {ss.s0};
                const double zz[1] = {z};
                if (p->symmetric && (rc = enqueue_dk(p, g, l0, np, z, ss.sm, ss.sn, 0, gs))) return rc;
                if ((rc = enqueue_couplings(p, g, l0, np, 1, sl, zz, gs))) return rc;
                if (p->symmetric && ((rc = enqueue_symm(p, g, l0, np, ss.s0, 0, gs)) ||
                                     (rc = enqueue_rhs(p, g, l0, np, 1, sl, gs))))
                    return rc;
            }
            const int sl[2] = {ss.sm, ss.sn};
            const double zz[2] = {zm, zn};
            if (p->symmetric && ((rc = enqueue_dk(p, g, l0, np, zm, ss.sm, ss.sn, 0, gs)) ||
                                 (rc = enqueue_dk(p, g, l0, np, zn, ss.sm, ss.sn, 1, gs))))
                return rc;
            if ((rc = enqueue_couplings(p, g, l0, np, 2, sl, zz, gs))) return rc;
            if (p->symmetric && ((rc = enqueue_symm(p, g, l0, np, ss.sm, 0, gs)) ||
                                 (rc = enqueue_symm(p, g, l0, np, ss.sn, 1, gs)) ||
                                 (rc = enqueue_rhs(p, g, l0, np, 2, sl, gs))))
                return rc;
            if (with_stages && !p->stage_all &&
                (rc = enqueue_stages(p, p->d_pm + p->pm_first[gi] + l0, np, g.m.N, ss, h, X, gs)))
                return rc;
        }
        if (fork) {
            WPCCC_HIP_CHECK(hipEventRecord(p->join_ev[gi], gs));
            WPCCC_HIP_CHECK(hipStreamWaitEvent(st, p->join_ev[gi], 0));
        }
    }
    // the stages of every group's paths in one launch each, after all couplings
    if (with_stages && p->stage_all &&
        (rc = enqueue_stages(p, p->d_pm, p->n_traj, p->N_max, ss, h, X, st, early1 ? 2 : 1)))
        return rc;
    return WPCCC_OK;
}

// One RK4 step z -> z + h of every path.
int enqueue_step(Plan2C* p, double2* X, double z, double h, hipStream_t st) {
    const StepSlots ss = step_slots(p, z);
    for (int s = 0; s < kSlots2C; ++s) p->slot_ok[s] = false;
    int rc;
    if ((rc = enqueue_step_slots(p, X, z, h, ss, st))) return rc;
    commit_slots(p, ss, z, h);
    return WPCCC_OK;
}

void drop_graphs(Plan2C* p) {
    for (int s = 0; s < kSlots2C; ++s) {
        if (p->gexec[s]) (void)hipGraphExecDestroy(p->gexec[s]);
        p->gexec[s] = nullptr;
    }
    for (auto& e : p->pexec) (void)hipGraphExecDestroy(e.second);
    p->pexec.clear();
    p->gX = nullptr;
}

// Slots of a pipelined step: it reads s0 (z), sm (z + h/2), sn (z + h) and
// forms the next step's couplings at z' + h'/2 and z' + h' (z' = z + h) in
// f1 and f2; the next step's slots are (sn, f1, f2, s0, sm).
struct PipeSlots {
    int s0, sm, sn, f1, f2;
};
int pipe_key(const PipeSlots& q) { return (((q.s0 * kSlots2C + q.sm) * kSlots2C + q.sn) * kSlots2C + q.f1) * kSlots2C + q.f2; }

// Graph step of the pipelined replay: the couplings of the next step on the
// group streams (one stream of its own for a one-group plan) beside this
// step's four stages on st; positions and step lengths from d_zh.
int enqueue_pipe_step(Plan2C* p, double2* X, const PipeSlots& q, hipStream_t st) {
    int rc;
    WPCCC_HIP_CHECK(hipEventRecord(p->pfork, st));
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        Group2C& g = p->groups[gi];
        hipStream_t gs = p->gstreams.empty() ? p->pstream : p->gstreams[gi];
        WPCCC_HIP_CHECK(hipStreamWaitEvent(gs, p->pfork, 0));
        const int npath = (int)g.paths.size();
        const int sl[2] = {q.f1, q.f2};
        const double zz[2] = {0.0, 0.0};   // read from d_zh
        if ((rc = enqueue_couplings(p, g, 0, npath, 2, sl, zz, gs)) || (rc = enqueue_rhs(p, g, 0, npath, 2, sl, gs)))
            return rc;
        WPCCC_HIP_CHECK(hipEventRecord(p->pjoin[gi], gs));
    }
    const StepSlots ss{true, q.s0, q.sm, q.sn};
    if ((rc = enqueue_stages(p, p->d_pm, p->n_traj, p->N_max, ss, 0.0, X, st))) return rc;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) WPCCC_HIP_CHECK(hipStreamWaitEvent(st, p->pjoin[gi], 0));
    return WPCCC_OK;
}

int capture_pipe_graph(Plan2C* p, double2* X, const PipeSlots& q, hipGraphExec_t* out) {
    *out = nullptr;
    if (!p->gcap) WPCCC_HIP_CHECK(hipStreamCreate(&p->gcap));
    WPCCC_HIP_CHECK(hipStreamBeginCapture(p->gcap, hipStreamCaptureModeRelaxed));
    const bool timing = p->timer->on;
    p->timer->on = false;
    p->capturing = true;
    p->zahead = 1;
    int rc = enqueue_pipe_step(p, X, q, p->gcap);
    if (rc == WPCCC_OK) rc = launched(launch_chunk_counter(p->d_step, 0, p->gcap), "k_chunk_counter");
    p->zahead = 0;
    p->capturing = false;
    p->timer->on = timing;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gcap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        *out = nullptr;
        set_error("graph instantiation failed: %s", hipGetErrorString(ei));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

// Capture the step that starts in slot s0 (its couplings there held) into
// gexec[s0]: positions and step length from d_zh at *d_step, which the
// last node advances.  Nothing runs during the capture.
int capture_step_graph(Plan2C* p, double2* X, int s0) {
    if (!p->gcap) WPCCC_HIP_CHECK(hipStreamCreate(&p->gcap));
    WPCCC_HIP_CHECK(hipStreamBeginCapture(p->gcap, hipStreamCaptureModeRelaxed));
    const bool timing = p->timer->on;
    p->timer->on = false;
    p->capturing = true;
    int rc = enqueue_step_slots(p, X, 0.0, 0.0, slots_with_start(s0, true), p->gcap);
    if (rc == WPCCC_OK) rc = launched(launch_chunk_counter(p->d_step, 0, p->gcap), "k_chunk_counter");
    p->capturing = false;
    p->timer->on = timing;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->gcap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    const hipError_t ei = hipGraphInstantiate(&p->gexec[s0], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
        p->gexec[s0] = nullptr;
        set_error("graph instantiation failed: %s", hipGetErrorString(ei));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

// d_zh with room for n entries of (z + h/2, z + h, h) (graphs that read the
// old array are dropped).
int reserve_zh(Plan2C* p, int n, hipStream_t st) {
    if (n <= p->zh_cap) return WPCCC_OK;
    if (p->zh_copied) WPCCC_HIP_CHECK(hipEventSynchronize(p->zh_copied));
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    drop_graphs(p);
    if (p->h_zh) (void)hipHostFree(p->h_zh);
    if (p->d_zh) (void)hipFree(p->d_zh);
    p->h_zh = nullptr;
    p->d_zh = nullptr;
    p->zh_cap = 0;
    WPCCC_HIP_CHECK(hipHostMalloc((void**)&p->h_zh, (size_t)3 * n * sizeof(double), 0));
    WPCCC_HIP_CHECK(hipMalloc((void**)&p->d_zh, (size_t)3 * n * sizeof(double)));
    p->bytes += (long long)3 * n * sizeof(double);
    if (!p->d_step) {
        WPCCC_HIP_CHECK(hipMalloc((void**)&p->d_step, sizeof(int)));
        p->bytes += sizeof(int);
    }
    if (!p->zh_copied) WPCCC_HIP_CHECK(hipEventCreateWithFlags(&p->zh_copied, hipEventDisableTiming));
    p->zh_cap = n;
    return WPCCC_OK;
}

// Pipelined replay of n >= 2 steps (stages over every group in one launch),
// per run of steps that each start where the previous one ended: the
// couplings of its first step launch by launch (those at z where not held),
// then graph steps, each the stages of step k beside the couplings of step
// k + 1 (PipeSlots), then the stages of its last step launch by launch.  The
// same kernels on the same data as enqueue_step, hence the same amplitudes;
// the stages no longer wait for the next positions' LU.
int propagate_pipe(Plan2C* p, const double* zgrid, int n_points, double2* X, hipStream_t st) {
    const int n_steps = n_points - 1;
    int rc;
    if ((rc = reserve_zh(p, n_steps, st))) return rc;
    // the staging buffer may still feed the previous call's copy
    WPCCC_HIP_CHECK(hipEventSynchronize(p->zh_copied));
    for (int i = 0; i < n_steps; ++i) {
        const double z = zgrid[i], h = zgrid[i + 1] - zgrid[i];
        p->h_zh[3 * i] = z + 0.5 * h;
        p->h_zh[3 * i + 1] = z + h;
        p->h_zh[3 * i + 2] = h;
    }
    WPCCC_HIP_CHECK(hipMemcpyAsync(p->d_zh, p->h_zh, (size_t)3 * n_steps * sizeof(double), hipMemcpyHostToDevice, st));
    WPCCC_HIP_CHECK(hipEventRecord(p->zh_copied, st));
    if ((rc = launched(launch_chunk_counter(p->d_step, 1, st), "k_chunk_counter"))) return rc;
    if (p->gX != X) drop_graphs(p);
    if (!p->pfork) {
        // the join events and the coupling stream first: pfork set means all exist
        while (p->pjoin.size() < p->groups.size()) {
            hipEvent_t ev = nullptr;
            WPCCC_HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            p->pjoin.push_back(ev);
        }
        if (p->gstreams.empty() && !p->pstream) WPCCC_HIP_CHECK(hipStreamCreate(&p->pstream));  // default priority
        WPCCC_HIP_CHECK(hipEventCreateWithFlags(&p->pfork, hipEventDisableTiming));
    }
    // segments of steps whose start point is the previous step's end point
    // exactly (z_k + h_k == z_(k+1) in floating point): a step that starts
    // elsewhere forms its couplings at z_(k+1), as enqueue_step does
    for (int i = 0; i < n_steps;) {
        int j = i;
        while (j + 1 < n_steps && zgrid[j] + (zgrid[j + 1] - zgrid[j]) == zgrid[j + 1]) ++j;
        // the couplings of step i (those at z_i where not held)
        const StepSlots s0 = step_slots(p, zgrid[i]);
        for (int k = 0; k < kSlots2C; ++k) p->slot_ok[k] = false;
        if ((rc = enqueue_step_slots(p, X, zgrid[i], zgrid[i + 1] - zgrid[i], s0, st, false))) return rc;
        PipeSlots q{s0.s0, s0.sm, s0.sn, -1, -1};
        for (int k = 0; k < kSlots2C; ++k)
            if (k != q.s0 && k != q.sm && k != q.sn) {
                if (q.f1 < 0) q.f1 = k;
                else if (q.f2 < 0) q.f2 = k;
            }
        // graph steps i .. j-1 (the device counter is the step index)
        for (int k = i; k < j; ++k) {
            const int key = pipe_key(q);
            hipGraphExec_t ex = nullptr;
            for (const auto& e : p->pexec)
                if (e.first == key) ex = e.second;
            if (!ex) {
                // the group streams take part in the capture: let them drain first
                WPCCC_HIP_CHECK(hipStreamSynchronize(st));
                if ((rc = capture_pipe_graph(p, X, q, &ex))) return rc;
                p->pexec.push_back({key, ex});
            }
            WPCCC_HIP_CHECK(hipGraphLaunch(ex, st));
            q = PipeSlots{q.sn, q.f1, q.f2, q.s0, q.sm};
        }
        p->gX = X;
        // the stages of step j; the slots then hold its three positions
        const double zl = zgrid[j], hl = zgrid[j + 1] - zl;
        const StepSlots sl{true, q.s0, q.sm, q.sn};
        if ((rc = enqueue_stages(p, p->d_pm, p->n_traj, p->N_max, sl, hl, X, st))) return rc;
        commit_slots(p, sl, zl, hl);
        if ((rc = launched(launch_chunk_counter(p->d_step, 0, st), "k_chunk_counter"))) return rc;
        i = j + 1;
    }
    return WPCCC_OK;
}

// Steps of zgrid by graph replays wherever the step's start point is held,
// launch by launch elsewhere (the first step of a run): the same slots, the
// same kernels on the same data as enqueue_step, hence the same amplitudes.
// With one stage launch over every group and the factored solves, the
// pipelined form above (with M = S^-1 H formed per point, its N^3 right-hand
// sides beside the next step's contractions measured slower than this form).
int propagate_graph(Plan2C* p, const double* zgrid, int n_points, double2* X, hipStream_t st) {
    const int n_steps = n_points - 1;
    if (p->stage_all && !p->explicit_m && n_steps >= 2) return propagate_pipe(p, zgrid, n_points, X, st);
    // which steps replay: the slot bookkeeping of the whole run, simulated
    double sz[kSlots2C];
    bool sok[kSlots2C];
    std::copy(p->slot_z, p->slot_z + kSlots2C, sz);
    std::copy(p->slot_ok, p->slot_ok + kSlots2C, sok);
    std::vector<int> start(n_steps);
    bool need[kSlots2C] = {};
    int n_rep = 0;
    for (int i = 0; i < n_steps; ++i) {
        const double z = zgrid[i], h = zgrid[i + 1] - zgrid[i];
        const StepSlots ss = step_slots(p, z);
        start[i] = ss.have0 ? ss.s0 : -1;
        if (ss.have0) {
            need[ss.s0] = true;
            ++n_rep;
        }
        commit_slots(p, ss, z, h);
    }
    std::copy(sz, sz + kSlots2C, p->slot_z);
    std::copy(sok, sok + kSlots2C, p->slot_ok);
    int rc;
    if ((rc = reserve_zh(p, n_rep, st))) return rc;
    if (n_rep > 0) {
        // the staging buffer may still feed the previous call's copy
        WPCCC_HIP_CHECK(hipEventSynchronize(p->zh_copied));
        int r = 0;
        for (int i = 0; i < n_steps; ++i) {
            if (start[i] < 0) continue;
            const double z = zgrid[i], h = zgrid[i + 1] - zgrid[i];
            p->h_zh[3 * r] = z + 0.5 * h;
            p->h_zh[3 * r + 1] = z + h;
            p->h_zh[3 * r + 2] = h;
            ++r;
        }
        WPCCC_HIP_CHECK(hipMemcpyAsync(p->d_zh, p->h_zh, (size_t)3 * n_rep * sizeof(double),
                                       hipMemcpyHostToDevice, st));
        WPCCC_HIP_CHECK(hipEventRecord(p->zh_copied, st));
        if ((rc = launched(launch_chunk_counter(p->d_step, 1, st), "k_chunk_counter"))) return rc;
        if (p->gX != X) drop_graphs(p);
        bool fresh = false;
        for (int s = 0; s < kSlots2C; ++s)
            if (need[s] && !p->gexec[s]) {
                if (!fresh) {
                    // the group streams take part in the capture: let them drain first
                    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
                    fresh = true;
                }
                if ((rc = capture_step_graph(p, X, s))) return rc;
            }
        p->gX = X;
    }
    for (int i = 0; i < n_steps; ++i) {
        const double z = zgrid[i], h = zgrid[i + 1] - zgrid[i];
        if (start[i] < 0) {
            if ((rc = enqueue_step(p, X, z, h, st))) return rc;
            continue;
        }
        const StepSlots ss = slots_with_start(start[i], true);
        for (int s = 0; s < kSlots2C; ++s) p->slot_ok[s] = false;
        WPCCC_HIP_CHECK(hipGraphLaunch(p->gexec[start[i]], st));
        commit_slots(p, ss, z, h);
    }
    return WPCCC_OK;
}

}  // namespace

int plan2c_create(const wpccc_basis_t* targets, const wpccc_basis_t* projectiles, int n_sets, int n_traj,
                  const int* set_of_traj, const double* b, const double* v, const wpccc_plan_opts& o,
                  KernelTimer* timer, hipStream_t st, Plan2C** out) {
    *out = nullptr;
    if (o.q_lower != WPCCC_Q_DAGGER && o.q_lower != WPCCC_Q_PRIOR) {
        set_error("wpccc_plan_create_2c: q_lower must be WPCCC_Q_DAGGER or WPCCC_Q_PRIOR");
        return WPCCC_EINVAL;
    }
    if (o.precision != WPCCC_FP64 && o.precision != WPCCC_MIXED) {
        set_error("wpccc_plan_create_2c: precision must be WPCCC_FP64 or WPCCC_MIXED");
        return WPCCC_EINVAL;
    }
    if (o.batched < 0 || o.batched > 2) {
        set_error("wpccc_plan_create_2c: batched must be 0, 1 or 2");
        return WPCCC_EINVAL;
    }
    if (o.symmetric != 0 && o.symmetric != 1) {
        set_error("wpccc_plan_create_2c: symmetric must be 0 or 1");
        return WPCCC_EINVAL;
    }
    if (o.symmetric && !(o.dz_sym == 0.0 || (o.dz_sym > 0.0 && o.dz_sym <= 0.01))) {
        set_error("wpccc_plan_create_2c: dz_sym must be 0 (1e-4) or in (0, 0.01]");
        return WPCCC_EINVAL;
    }
    if (o.symmetric && (o.precision == WPCCC_MIXED || o.graph)) {
        set_error("wpccc_plan_create_2c: the symmetric form is FP64 and launched kernel by kernel");
        return WPCCC_ENOTSUP;
    }
    if (o.solve != WPCCC_SOLVE_FACTORED && o.solve != WPCCC_SOLVE_EXPLICIT) {
        set_error("wpccc_plan_create_2c: solve must be WPCCC_SOLVE_FACTORED or WPCCC_SOLVE_EXPLICIT");
        return WPCCC_EINVAL;
    }
    if (o.n_eta < 4 || o.n_eta > 1024 || o.n_tau < 4 || o.n_tau > 4096) {
        set_error("wpccc_plan_create_2c: n_eta must be in [4, 1024] and n_tau in [4, 4096]");
        return WPCCC_EINVAL;
    }
    for (int s = 0; s < n_sets; ++s)
        if (!targets[s] || !projectiles[s]) {
            set_error("wpccc_plan_create_2c: NULL basis in set %d", s);
            return WPCCC_EINVAL;
        }
    for (int j = 0; j < n_traj; ++j) {
        if (set_of_traj[j] < 0 || set_of_traj[j] >= n_sets) {
            set_error("wpccc_plan_create_2c: path %d names set %d of %d", j, set_of_traj[j], n_sets);
            return WPCCC_EINVAL;
        }
        if (!(b[j] > 0.0) || !(v[j] > 0.0) || !std::isfinite(b[j]) || !std::isfinite(v[j])) {
            set_error("wpccc_plan_create_2c: path %d needs finite b > 0 and v > 0", j);
            return WPCCC_EINVAL;
        }
    }
    int rc;
    for (int s = 0; s < n_sets; ++s) {
        if ((rc = check_basis(targets[s]->hb, "target"))) return rc;
        if ((rc = check_basis(projectiles[s]->hb, "projectile"))) return rc;
        if (targets[s]->hb.n_states + projectiles[s]->hb.n_states > kLUMaxN) {
            set_error("wpccc_plan_create_2c: set %d has %d states; at most %d are supported", s,
                      targets[s]->hb.n_states + projectiles[s]->hb.n_states, kLUMaxN);
            return WPCCC_ENOTSUP;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("wpccc_plan_create_2c: no HIP device available");
        return WPCCC_EHIP;
    }
    Plan2C* p = new (std::nothrow) Plan2C;
    if (!p) {
        set_error("wpccc_plan_create_2c: out of host memory");
        return WPCCC_ENOMEM;
    }
    p->timer = timer;
    p->n_traj = n_traj;
    p->batched = o.batched ? 1 : 0;
    p->stage_all = o.batched == 1;
    p->q_prior = o.q_lower == WPCCC_Q_PRIOR;
    p->mixed = o.precision == WPCCC_MIXED;
    p->explicit_m = o.solve == WPCCC_SOLVE_EXPLICIT;
    p->use_graph = o.graph != 0;
    p->symmetric = o.symmetric != 0;
    if (o.dz_sym != 0.0) p->dz_sym = o.dz_sym;
    p->n_eta = o.n_eta;
    p->n_tau = o.n_tau;
    p->b.assign(b, b + n_traj);
    p->v.assign(v, v + n_traj);
    p->group_of.assign(n_traj, -1);
    p->local_of.assign(n_traj, -1);
    int maxN = 0;
    for (int s = 0; s < n_sets; ++s) {
        Group2C g;
        g.tb = &targets[s]->hb;
        g.pb = &projectiles[s]->hb;
        for (int j = 0; j < n_traj; ++j)
            if (set_of_traj[j] == s) {
                p->group_of[j] = (int)p->groups.size();
                p->local_of[j] = (int)g.paths.size();
                g.paths.push_back(j);
            }
        if (g.paths.empty()) continue;
        maxN = std::max(maxN, g.tb->n_states + g.pb->n_states);
        p->groups.push_back(g);
    }
    p->n_pad = (maxN + 7) & ~7;
    auto fail = [&](int code) {
        plan2c_destroy(p);
        return code;
    };
    for (Group2C& g : p->groups)
        if ((rc = build_group(p, g, st))) return fail(rc);
    // stage descriptors, group by group
    {
        std::vector<PathMats> pm;
        for (Group2C& g : p->groups) {
            p->pm_first.push_back((int)pm.size());
            const size_t NN = (size_t)g.m.N * g.m.N;
            for (size_t l = 0; l < g.paths.size(); ++l) {
                PathMats e{};
                e.N = g.m.N;
                e.path = g.paths[l];
                e.H = (p->explicit_m ? g.d_M : g.d_H) + l * kSlots2C * NN;
                e.LU = g.d_LU + l * kSlots2C * NN;
                e.perm = p->explicit_m ? nullptr : g.d_perm + l * kSlots2C * g.m.N;
                pm.push_back(e);
            }
            p->N_max = std::max(p->N_max, g.m.N);
        }
        if ((rc = dev_alloc(&p->d_pm, pm.size(), p->bytes))) return fail(rc);
        if ((rc = upload(p->d_pm, pm.data(), pm.size() * sizeof(PathMats), st))) return fail(rc);
    }
    std::vector<double> xl, wl, tl, wt;
    gauss_laguerre_scaled(p->n_eta, xl, wl);
    gauss_legendre(p->n_tau, tl, wt);
    long long& tot = p->bytes;
    if ((rc = dev_alloc(&p->d_b, (size_t)n_traj, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_v, (size_t)n_traj, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_flag, 4, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_Ua, (size_t)n_traj * p->n_pad, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_Ub, (size_t)n_traj * p->n_pad, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_Xacc, (size_t)n_traj * p->n_pad, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_Y, (size_t)n_traj * p->n_pad, tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_xlag, xl.size(), tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_wlag, wl.size(), tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_tleg, tl.size(), tot))) return fail(rc);
    if ((rc = dev_alloc(&p->d_wleg, wt.size(), tot))) return fail(rc);
    if ((rc = upload(p->d_b, b, n_traj * sizeof(double), st))) return fail(rc);
    if ((rc = upload(p->d_v, v, n_traj * sizeof(double), st))) return fail(rc);
    if ((rc = upload(p->d_xlag, xl.data(), xl.size() * sizeof(double), st))) return fail(rc);
    if ((rc = upload(p->d_wlag, wl.data(), wl.size() * sizeof(double), st))) return fail(rc);
    if ((rc = upload(p->d_tleg, tl.data(), tl.size() * sizeof(double), st))) return fail(rc);
    if ((rc = upload(p->d_wleg, wt.data(), wt.size() * sizeof(double), st))) return fail(rc);
    hipError_t e = hipMemsetAsync(p->d_flag, 0, 4 * sizeof(int), st);
    if (e == hipSuccess && p->groups.size() > 1) {
        e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
        for (size_t gi = 0; gi < p->groups.size() && e == hipSuccess; ++gi) {
            hipStream_t gs = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreate(&gs);  // default priority
            if (e == hipSuccess) {
                p->gstreams.push_back(gs);
                e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                if (e == hipSuccess) p->join_ev.push_back(ev);
            }
        }
        if (e != hipSuccess || p->join_ev.size() != p->groups.size()) {
            // fall back to the caller's stream only
            for (hipStream_t gs : p->gstreams) (void)hipStreamDestroy(gs);
            for (hipEvent_t ev : p->join_ev) (void)hipEventDestroy(ev);
            p->gstreams.clear();
            p->join_ev.clear();
            (void)hipGetLastError();
            e = hipSuccess;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error("wpccc_plan_create_2c: device setup failed: %s", hipGetErrorString(e));
        return fail(WPCCC_EHIP);
    }
    *out = p;
    return WPCCC_OK;
}

void plan2c_destroy(Plan2C* p) {
    if (!p) return;
    if (p->zh_copied) {
        (void)hipEventSynchronize(p->zh_copied);
        (void)hipEventDestroy(p->zh_copied);
    }
    drop_graphs(p);
    if (p->gcap) (void)hipStreamDestroy(p->gcap);
    if (p->pstream) {
        (void)hipStreamSynchronize(p->pstream);
        (void)hipStreamDestroy(p->pstream);
    }
    if (p->pfork) (void)hipEventDestroy(p->pfork);
    for (hipEvent_t ev : p->pjoin) (void)hipEventDestroy(ev);
    if (p->h_zh) (void)hipHostFree(p->h_zh);
    if (p->d_zh) (void)hipFree(p->d_zh);
    if (p->d_step) (void)hipFree(p->d_step);
    for (hipStream_t gs : p->gstreams) {
        (void)hipStreamSynchronize(gs);
        (void)hipStreamDestroy(gs);
    }
    for (hipEvent_t ev : p->join_ev) (void)hipEventDestroy(ev);
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    for (Group2C& g : p->groups) free_group(g);
    void* bufs[] = {p->d_b,    p->d_v,    p->d_flag, p->d_Ua,   p->d_Ub,  p->d_Xacc,
                    p->d_Y,    p->d_xlag, p->d_wlag, p->d_tleg, p->d_wleg, p->d_pm};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    delete p;
}

int plan2c_info(Plan2C* p, int* n_traj, int* n_states, int* n_pad, long long* bytes) {
    int maxN = 0;
    for (const Group2C& g : p->groups) maxN = std::max(maxN, g.m.N);
    if (n_traj) *n_traj = p->n_traj;
    if (n_states) *n_states = maxN;
    if (n_pad) *n_pad = p->n_pad;
    if (bytes) *bytes = p->bytes;
    return WPCCC_OK;
}

int plan2c_path_info(Plan2C* p, int j, int* n_states, int* n_target) {
    if (j < 0 || j >= p->n_traj) {
        set_error("wpccc_plan_path_info: path index out of range");
        return WPCCC_EINVAL;
    }
    const Group2C& g = p->groups[p->group_of[j]];
    if (n_states) *n_states = g.m.N;
    if (n_target) *n_target = g.m.NT;
    return WPCCC_OK;
}

int plan2c_status(Plan2C* p, hipStream_t st) {
    int flag[4] = {0, 0, 0, 0};
    WPCCC_HIP_CHECK(hipMemcpyAsync(flag, p->d_flag, sizeof flag, hipMemcpyDeviceToHost, st));
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    WPCCC_HIP_CHECK(hipMemsetAsync(p->d_flag, 0, sizeof flag, st));
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    if (flag[1]) {
        set_error("overlap matrix S singular on path %d (zero pivot in column %d)", flag[1] - 1, flag[2]);
        return WPCCC_ESINGULAR;
    }
    if (flag[0]) {
        set_error("non-finite amplitude detected during propagation");
        return WPCCC_ENUMERIC;
    }
    return WPCCC_OK;
}

int plan2c_couplings(Plan2C* p, int j, double z, void* H, void* S, hipStream_t st) {
    if (j < 0 || j >= p->n_traj) {
        set_error("wpccc_couplings: path index out of range");
        return WPCCC_EINVAL;
    }
    if (!S) {
        set_error("wpccc_couplings: S_dev is required for a two-centre plan");
        return WPCCC_EINVAL;
    }
    if (!(std::sqrt(p->b[j] * p->b[j] + z * z) > 0.0)) {
        set_error("wpccc_couplings: R = 0");
        return WPCCC_EINVAL;
    }
    Group2C& g = p->groups[p->group_of[j]];
    const int l = p->local_of[j];
    for (int s = 0; s < kSlots2C; ++s) p->slot_ok[s] = false;
    const int sl[1] = {0};
    const double zz[1] = {z};
    int rc;
    if (p->symmetric && (rc = enqueue_dk(p, g, l, 1, z, 1, 2, 0, st))) return rc;
    if ((rc = enqueue_couplings(p, g, l, 1, 1, sl, zz, st))) return rc;
    if (p->symmetric && (rc = enqueue_symm(p, g, l, 1, 0, 0, st))) return rc;
    const size_t NN = (size_t)g.m.N * g.m.N;
    const size_t off = (size_t)l * kSlots2C * NN;
    WPCCC_HIP_CHECK(hipMemcpyAsync(H, g.d_H + off, NN * sizeof(double2), hipMemcpyDeviceToDevice, st));
    return launched(launch_transpose_copy(g.d_S + off, (double2*)S, g.m.N, st), "k_transpose_copy");
}

int plan2c_step(Plan2C* p, void* X, double z, double h, hipStream_t st) {
    if (hits_origin(p, z) || hits_origin(p, z + 0.5 * h) || hits_origin(p, z + h)) {
        set_error("wpccc_step: R = 0 on the step");
        return WPCCC_EINVAL;
    }
    return enqueue_step(p, (double2*)X, z, h, st);
}

int plan2c_propagate(Plan2C* p, const double* zgrid, int n_points, void* Xv, void* P, void* norm, hipStream_t st) {
    for (int i = 0; i < n_points; ++i)
        if (hits_origin(p, zgrid[i]) || (i + 1 < n_points && hits_origin(p, 0.5 * (zgrid[i] + zgrid[i + 1])))) {
            set_error("wpccc_propagate: R = 0 on the grid");
            return WPCCC_EINVAL;
        }
    double2* X = (double2*)Xv;
    int rc;
    if (p->use_graph && !p->timer->on) {
        if ((rc = propagate_graph(p, zgrid, n_points, X, st))) return rc;
    } else {
        for (int i = 0; i + 1 < n_points; ++i)
            if ((rc = enqueue_step(p, X, zgrid[i], zgrid[i + 1] - zgrid[i], st))) return rc;
    }
    if (!P && !norm) return WPCCC_OK;
    const double zl = zgrid[n_points - 1];
    for (Group2C& g : p->groups) {
        const int npath = (int)g.paths.size();
        int slot = find_slot(p, zl);
        if (slot < 0) {
            // S at the last point for every path of the group
            slot = 0;
            for (int s = 0; s < kSlots2C; ++s) p->slot_ok[s] = false;
            const int sl[1] = {0};
            const double zz[1] = {zl};
            const int chunk = std::max(1, g.max_jobs);
            for (int l0 = 0; l0 < npath; l0 += chunk)
                if ((rc = enqueue_couplings(p, g, l0, std::min(chunk, npath - l0), 1, sl, zz, st, false))) return rc;
        }
        if ((rc = timed(p, k2cFinish, [&](const LaunchEv& ev) {
                 return launch_2c_finish(X, g.d_S, g.m.N, p->n_pad, g.d_paths, npath, slot, (double*)P,
                                         (double*)norm, st, ev);
             })))
            return rc;
    }
    return WPCCC_OK;
}

// A X = B for `batch` complex n x n systems with n right-hand sides: the LU
// panels with partial pivoting over every column, then k_lu_rhs.  The
// kernels address their matrices with the plan's slot stride, so A and B
// are staged at that stride in buffers of this call.
int lu_solve_batched(int n, int batch, const void* A, const void* B, void* X, hipStream_t st) {
    if (n < 1 || n > kLUMaxN || batch < 1 || !A || !B || !X) {
        set_error("wpccc_zgesv_batched: need 1 <= n <= %d, batch >= 1 and non-NULL matrices", kLUMaxN);
        return WPCCC_EINVAL;
    }
    const size_t NN = (size_t)n * n, per = (size_t)kSlots2C * NN;
    double2 *lu = nullptr, *hb = nullptr, *mb = nullptr;
    int *piv = nullptr, *perm = nullptr, *paths = nullptr, *flag = nullptr;
    int rc = WPCCC_OK;
    long long tot = 0;
    std::vector<int> ids(batch);
    for (int i = 0; i < batch; ++i) ids[i] = i;
    int hflag[4] = {0, 0, 0, 0};
    auto run = [&]() -> int {
        int r;
        if ((r = dev_alloc(&lu, per * batch, tot)) || (r = dev_alloc(&hb, per * batch, tot)) ||
            (r = dev_alloc(&mb, per * batch, tot)) || (r = dev_alloc(&piv, (size_t)kSlots2C * n * batch, tot)) ||
            (r = dev_alloc(&perm, (size_t)kSlots2C * n * batch, tot)) || (r = dev_alloc(&paths, batch, tot)) ||
            (r = dev_alloc(&flag, 4, tot)))
            return r;
        if ((r = upload(paths, ids.data(), batch * sizeof(int), st))) return r;
        WPCCC_HIP_CHECK(hipMemsetAsync(flag, 0, 4 * sizeof(int), st));
        WPCCC_HIP_CHECK(hipMemcpy2DAsync(lu, per * sizeof(double2), A, NN * sizeof(double2), NN * sizeof(double2),
                                         batch, hipMemcpyDeviceToDevice, st));
        WPCCC_HIP_CHECK(hipMemcpy2DAsync(hb, per * sizeof(double2), B, NN * sizeof(double2), NN * sizeof(double2),
                                         batch, hipMemcpyDeviceToDevice, st));
        LUStepArgs a{};
        a.N = n;
        a.jobs.path0 = 0;
        a.jobs.n_sub = 1;
        a.LU = lu;
        a.piv = piv;
        a.perm = perm;
        a.paths = paths;
        a.flag = flag;
        a.skip_mode = 0;
        const int pw = lu_panel_width(n);
        for (int k0 = 0; k0 < n; k0 += pw) {
            a.k0 = k0;
            a.nb = std::min(pw, n - k0);
            if ((r = launched(launch_lu_panel(a, batch, st), "k_lu_panel")) ||
                (r = launched(launch_lu_swap_trsm(a, batch, st), "k_lu_swap_trsm")) ||
                (r = launched(launch_lu_update(a, batch, st), "k_lu_update")))
                return r;
        }
        RhsArgs ra{};
        ra.N = n;
        ra.jobs = a.jobs;
        ra.LU = lu;
        ra.perm = perm;
        ra.H = hb;
        ra.M = mb;
        if ((r = launched(launch_lu_rhs(ra, batch, st), "k_lu_rhs"))) return r;
        WPCCC_HIP_CHECK(hipMemcpy2DAsync(X, NN * sizeof(double2), mb, per * sizeof(double2), NN * sizeof(double2),
                                         batch, hipMemcpyDeviceToDevice, st));
        WPCCC_HIP_CHECK(hipMemcpyAsync(hflag, flag, sizeof hflag, hipMemcpyDeviceToHost, st));
        WPCCC_HIP_CHECK(hipStreamSynchronize(st));
        return WPCCC_OK;
    };
    rc = run();
    if (rc != WPCCC_OK) (void)hipStreamSynchronize(st);
    void* bufs[] = {lu, hb, mb, piv, perm, paths, flag};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    if (rc != WPCCC_OK) return rc;
    if (hflag[1]) {
        set_error("wpccc_zgesv_batched: matrix %d is singular (zero pivot in column %d)", hflag[1] - 1, hflag[2]);
        return WPCCC_ESINGULAR;
    }
    return WPCCC_OK;
}

}  // namespace wpccc

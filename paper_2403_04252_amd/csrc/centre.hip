// Device tables of one centre's basis (setup, once per basis and plan).
//
// For the Eq. D1 couplings of this centre's states:
//   * the row layout of the radial integrals (see plan.h) and, per entry, the
//     partial radial moments (A_k, B_(k+1)) on every grid node (k_moments);
//   * lambda of every Frow column and the (block start, width, state offset)
//     of every G column;
//   * the Eq. D1 angular coefficients c(l'm', lm, lambda) with the index of
//     the Pbar_lambda^|mu| they multiply;
//   * energies per state and per radial function.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "plan.h"

namespace wpccc {

int dev_alloc_bytes(void** p, size_t bytes, long long& total) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        *p = nullptr;
        return e == hipErrorOutOfMemory ? WPCCC_ENOMEM : WPCCC_EHIP;
    }
    total += (long long)bytes;
    return WPCCC_OK;
}

int launched(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

namespace {

// number of multipoles lambda coupling l and l' (|l-l'|..l+l' step 2)
inline int n_lambda(int l, int lp) { return std::min(l, lp) + 1; }

// first column of block (l, lambda) in the l' row layouts (Frow / G)
void block_columns(const Meta& m, int lp, int l, int lam, int& e0, int& g0) {
    e0 = 0;
    g0 = 0;
    for (int ll = 0; ll < l; ++ll) {
        e0 += n_lambda(ll, lp) * m.n_l[ll];
        g0 += n_lambda(ll, lp) * (2 * ll + 1);
    }
    const int k = (lam - std::abs(l - lp)) / 2;
    e0 += k * m.n_l[l];
    g0 += k * (2 * l + 1);
}

}  // namespace

void centre_free(Centre& c) {
    void* bufs[] = {c.d_meta,   c.d_eps,  c.d_gcoef, c.d_rad_eps, c.d_col_lam,
                    c.d_gpb,    c.d_st_rad, c.d_st_xs, c.d_gcol,  c.d_tab, c.d_tab32, c.d_ftab};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    c = Centre{};
}

void model_blocks(const HostBasis& hb, double a, double c, std::vector<double>& va, std::vector<double>& vc) {
    va.clear();
    vc.clear();
    for (int l = 0; l <= hb.spec.l_max; ++l) {
        const int nl = hb.n_l[l];
        for (int np = 0; np < nl; ++np)
            for (int n = 0; n < nl; ++n) {
                const double* fp = hb.phi.data() + (size_t)(hb.rad_off[l] + np) * (hb.n_r + 1);
                const double* f = hb.phi.data() + (size_t)(hb.rad_off[l] + n) * (hb.n_r + 1);
                double sa = 0.0, sc = 0.0;
                for (int i = 1; i <= hb.n_r; ++i) {
                    const double r = hb.r[i], e = std::exp(-c * r) * hb.w[i] * fp[i] * f[i];
                    sa += r * e;
                    sc += r * r * e;
                }
                va.push_back(-sa);
                vc.push_back(a * sc);
            }
    }
}

int centre_build(const HostBasis& hb, hipStream_t st, Centre& c, double model_a, double model_c, double Zp,
                 int form) {
    if (hb.spec.l_max > kMaxL) {
        set_error("basis l_max %d exceeds %d", hb.spec.l_max, kMaxL);
        return WPCCC_EINVAL;
    }
    const int N = hb.n_states;
    Meta& m = c.meta;
    m.l_max = hb.spec.l_max;
    m.lam_max = 2 * m.l_max;
    m.n_r = hb.n_r;
    m.n_f = hb.n_f;
    m.n_states = N;
    m.r_max = hb.spec.r_max;
    for (int l = 0; l <= kMaxL; ++l) {
        m.n_l[l] = l <= m.l_max ? hb.n_l[l] : 0;
        m.state_off[l] = l <= m.l_max ? hb.state_off[l] : N;
        m.rad_off[l] = l <= m.l_max ? hb.rad_off[l] : hb.n_f;
    }
    // x' in LDS: rows (l, q) of N_l values at an odd stride (in 16-byte
    // units), so that lanes reading different q of one l hit different banks
    m.n_xs = 0;
    for (int l = 0; l <= kMaxL; ++l) {
        m.xs_off[l] = m.n_xs;
        m.xs_stride[l] = 0;
        if (l > m.l_max) continue;
        m.xs_stride[l] = m.n_l[l] | 1;
        m.n_xs += (2 * l + 1) * m.xs_stride[l];
    }
    std::vector<int> st_xs((size_t)N);
    for (int l = 0; l <= m.l_max; ++l)
        for (int q = 0; q <= 2 * l; ++q)
            for (int n = 0; n < m.n_l[l]; ++n)
                st_xs[(size_t)m.state_off[l] + q * m.n_l[l] + n] = m.xs_off[l] + q * m.xs_stride[l] + n;
    m.n_frow = m.n_g = m.n_chunks = m.n_cols = m.n_gcols = 0;
    for (int lp = 0; lp <= kMaxL; ++lp) {
        m.nV[lp] = m.gcols[lp] = 0;
        m.frow_off[lp] = m.n_frow;
        m.g_off[lp] = m.n_g;
        m.col_off[lp] = m.n_cols;
        m.gcol_off[lp] = m.n_gcols;
        if (lp > m.l_max) continue;
        for (int l = 0; l <= m.l_max; ++l) {
            m.nV[lp] += n_lambda(l, lp) * m.n_l[l];
            m.gcols[lp] += n_lambda(l, lp) * (2 * l + 1);
        }
        m.n_frow += m.n_l[lp] * m.nV[lp];
        m.n_g += (2 * lp + 1) * m.gcols[lp];
        m.n_cols += m.nV[lp];
        m.n_gcols += m.gcols[lp];
        m.n_chunks += (m.n_l[lp] + kRowsPerBlock - 1) / kRowsPerBlock;
    }
    // Frow entries (a, b, lambda) in row layout; column lambda and G column maps
    std::vector<int> da, db, dl, col_lam;
    std::vector<int2> gcol;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        std::vector<int> lam_of_col, a_off_of_col;
        for (int l = 0; l <= m.l_max; ++l)
            for (int lam = std::abs(l - lp); lam <= l + lp; lam += 2) {
                int e0, g0;
                block_columns(m, lp, l, lam, e0, g0);
                for (int n = 0; n < m.n_l[l]; ++n) {
                    lam_of_col.push_back(lam);
                    a_off_of_col.push_back(hb.rad_off[l] + n);
                }
                for (int q = 0; q <= 2 * l; ++q)
                    gcol.push_back(gcol_pack(e0, m.n_l[l], m.xs_off[l] + q * m.xs_stride[l]));
            }
        col_lam.insert(col_lam.end(), lam_of_col.begin(), lam_of_col.end());
        for (int np = 0; np < m.n_l[lp]; ++np)
            for (int e = 0; e < m.nV[lp]; ++e) {
                da.push_back(hb.rad_off[lp] + np);
                db.push_back(a_off_of_col[e]);
                dl.push_back(lam_of_col[e]);
            }
    }
    if ((int)da.size() != m.n_frow || (int)col_lam.size() != m.n_cols || (int)gcol.size() != m.n_gcols) {
        set_error("internal layout mismatch in the centre tables");
        return WPCCC_EINVAL;
    }
    // angular factors: c(l'm', lm, lambda) = -sqrt((2l+1)/(2l'+1)) C^{l'0}_{lam 0 l 0}
    // C^{l'm'}_{lam mu l m}, mu = m'-m, times (-1)^mu for mu < 0, so that
    // c * Pbar_lam^|mu| = -sqrt((2l+1)(lam-mu)!/((2l'+1)(lam+mu)!)) C C P_lam^mu (Eq. D1).
    std::vector<double> gcoef((size_t)m.n_g, 0.0);
    std::vector<int> gpb((size_t)m.n_g, -1);
    for (int lp = 0; lp <= m.l_max; ++lp)
        for (int qp = 0; qp <= 2 * lp; ++qp) {
            const int mp = qp - lp;
            for (int l = 0; l <= m.l_max; ++l)
                for (int lam = std::abs(l - lp); lam <= l + lp; lam += 2) {
                    int e0, g0;
                    block_columns(m, lp, l, lam, e0, g0);
                    for (int q = 0; q <= 2 * l; ++q) {
                        const int mm = q - l, mu = mp - mm;
                        const size_t idx = (size_t)m.g_off[lp] + (size_t)qp * m.gcols[lp] + g0 + q;
                        if (std::abs(mu) > lam) continue;
                        double cf = -std::sqrt((2.0 * l + 1.0) / (2.0 * lp + 1.0)) *
                                    clebsch_gordan(lam, 0, l, 0, lp, 0) * clebsch_gordan(lam, mu, l, mm, lp, mp);
                        if (cf == 0.0) continue;
                        if (mu < 0 && (mu % 2)) cf = -cf;
                        gcoef[idx] = cf;
                        gpb[idx] = pb_index(lam, std::abs(mu));
                    }
                }
        }
    // phi transposed [n_r+1][n_f]
    std::vector<double> phiT((size_t)(hb.n_r + 1) * hb.n_f);
    for (int a = 0; a < hb.n_f; ++a)
        for (int i = 0; i <= hb.n_r; ++i) phiT[(size_t)i * hb.n_f + a] = hb.phi[(size_t)a * (hb.n_r + 1) + i];

    long long& tot = c.bytes;
    int rc = WPCCC_OK;
    auto A = [&](int r) {
        if (rc == WPCCC_OK) rc = r;
    };
    A(dev_alloc(&c.d_meta, 1, tot));
    A(dev_alloc(&c.d_eps, (size_t)N, tot));
    A(dev_alloc(&c.d_st_rad, (size_t)N, tot));
    A(dev_alloc(&c.d_st_xs, (size_t)N, tot));
    A(dev_alloc(&c.d_rad_eps, (size_t)m.n_f, tot));
    A(dev_alloc(&c.d_gcoef, (size_t)m.n_g, tot));
    A(dev_alloc(&c.d_gpb, (size_t)m.n_g, tot));
    A(dev_alloc(&c.d_col_lam, (size_t)m.n_cols, tot));
    A(dev_alloc(&c.d_gcol, (size_t)m.n_gcols, tot));
    A(dev_alloc(&c.d_tab, (size_t)(m.n_r + 1) * m.n_frow, tot));
    double *d_r = nullptr, *d_w = nullptr, *d_phiT = nullptr;
    int *d_da = nullptr, *d_db = nullptr, *d_dl = nullptr;
    long long tmp = 0;
    A(dev_alloc(&d_r, hb.r.size(), tmp));
    A(dev_alloc(&d_w, hb.w.size(), tmp));
    A(dev_alloc(&d_phiT, phiT.size(), tmp));
    A(dev_alloc(&d_da, da.size(), tmp));
    A(dev_alloc(&d_db, db.size(), tmp));
    A(dev_alloc(&d_dl, dl.size(), tmp));
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (rc == WPCCC_OK && e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(c.d_meta, &c.meta, sizeof(Meta));
    up(c.d_eps, hb.eps.data(), (size_t)N * sizeof(double));
    up(c.d_st_rad, hb.st_i.data(), (size_t)N * sizeof(int));
    up(c.d_st_xs, st_xs.data(), (size_t)N * sizeof(int));
    up(c.d_rad_eps, hb.rad_eps.data(), (size_t)m.n_f * sizeof(double));
    up(c.d_gcoef, gcoef.data(), gcoef.size() * sizeof(double));
    up(c.d_gpb, gpb.data(), gpb.size() * sizeof(int));
    up(c.d_col_lam, col_lam.data(), col_lam.size() * sizeof(int));
    up(c.d_gcol, gcol.data(), gcol.size() * sizeof(int2));
    up(d_r, hb.r.data(), hb.r.size() * sizeof(double));
    up(d_w, hb.w.data(), hb.w.size() * sizeof(double));
    up(d_phiT, phiT.data(), phiT.size() * sizeof(double));
    up(d_da, da.data(), da.size() * sizeof(int));
    up(d_db, db.data(), db.size() * sizeof(int));
    up(d_dl, dl.data(), dl.size() * sizeof(int));
    if (rc == WPCCC_OK && e == hipSuccess)
        e = launch_moments(d_r, d_w, d_phiT, d_da, d_db, d_dl, m.n_r, m.n_f, m.n_frow, c.d_tab, st);
    // model potential: -DeltaV / Zp on the lambda = 0 moments B of the equal-l
    // blocks (D = Zp sum G F with G = -1 for lambda = 0, l = l', m = m')
    std::vector<int> sh_idx;
    std::vector<double> sh_val;
    int* d_sidx = nullptr;
    double* d_sval = nullptr;
    if (model_a != 0.0) {
        std::vector<double> va, vc;
        model_blocks(hb, model_a, model_c, va, vc);
        size_t vo = 0;
        for (int l = 0; l <= m.l_max; ++l) {
            int e0, g0;
            block_columns(m, l, l, 0, e0, g0);
            const int nl = m.n_l[l];
            for (int np = 0; np < nl; ++np)
                for (int n = 0; n < nl; ++n) {
                    sh_idx.push_back(m.frow_off[l] + np * m.nV[l] + e0 + n);
                    sh_val.push_back(-model_a * va[vo + (size_t)np * nl + n] / Zp);
                }
            vo += (size_t)nl * nl;
        }
        A(dev_alloc(&d_sidx, sh_idx.size(), tmp));
        A(dev_alloc(&d_sval, sh_val.size(), tmp));
        up(d_sidx, sh_idx.data(), sh_idx.size() * sizeof(int));
        up(d_sval, sh_val.data(), sh_val.size() * sizeof(double));
        if (rc == WPCCC_OK && e == hipSuccess)
            e = launch_table_shift(c.d_tab, m.n_frow, m.n_r, d_sidx, d_sval, (int)sh_idx.size(), st);
    }
    if (form != kRadialMoments) {
        // the scaled FP32 form or the node values replace the FP64 table (after the model shift)
        if (form == kRadialMoments32) A(dev_alloc(&c.d_tab32, (size_t)(m.n_r + 1) * m.n_frow, tot));
        else A(dev_alloc(&c.d_ftab, (size_t)(m.n_r + 1) * m.n_frow, tot));
        if (rc == WPCCC_OK && e == hipSuccess)
            e = form == kRadialMoments32 ? launch_table_f32(c.d_tab, d_dl, m.n_frow, m.n_r, m.r_max, c.d_tab32, st)
                                         : launch_table_nodes(c.d_tab, d_dl, m.n_frow, m.n_r, m.r_max, c.d_ftab, st);
        if (rc == WPCCC_OK && e == hipSuccess) e = hipStreamSynchronize(st);
        if (rc == WPCCC_OK && e == hipSuccess) {
            (void)hipFree(c.d_tab);
            c.d_tab = nullptr;
            tot -= (long long)((size_t)(m.n_r + 1) * m.n_frow * sizeof(double2));
        }
    }
    if (rc == WPCCC_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    void* tq[] = {d_r, d_w, d_phiT, d_da, d_db, d_dl, d_sidx, d_sval};
    for (void* x : tq)
        if (x) (void)hipFree(x);
    if (rc == WPCCC_OK && e != hipSuccess) {
        set_error("centre table setup failed: %s", hipGetErrorString(e));
        rc = WPCCC_EHIP;
    }
    if (rc != WPCCC_OK) centre_free(c);
    return rc;
}

}  // namespace wpccc

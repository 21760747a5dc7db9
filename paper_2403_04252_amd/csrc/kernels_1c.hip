// HIP kernels of the one-centre path on gfx950 (64-wide waves, FP64 VALU).
//
// One RK4 stage of Algorithm 1 for every path of the batch is one launch of
// k_stage: from (b, z, v) and the basis tables it forms, per workgroup, the
// part of M(z) = -(i/v) Zp D_T(b, z) it needs and applies it to the stage
// input, then writes the RK4 combination of that stage.  k_chunk runs the
// same stages for up to 64 steps in one persistent launch (per-path
// barriers between stages); k_apply applies M or its derivatives for the
// adjoint.  D_T (Eq. D1) is
// never formed: its (l'm', lm) block is sum_lambda c Pbar_lambda^|m'-m| F_lambda
// with F_lambda the N_l' x N_l matrix of Eq. D2 radial integrals, so
//   y_{l'm'}[n'] = sum_{l, lambda, q} G_l'[m'][(l,lambda), q] sum_n F_l'[n'][(l,lambda), n] x'_{l q n}
// with x' = conj(phase) u (interaction picture).
//
// Radial integrals at the exact R.  For the grid quadrature of Eq. D2
//   F(R) = sum_i w_i r_i^2 f_a f_b min(r_i,R)^lam / max(r_i,R)^(lam+1)
//        = R^-(lam+1) A_k + R^lam B_(k+1),
//   A_k = sum_{i<=k} w_i r_i^(2+lam) f_a f_b,   B_k = sum_{i>=k} w_i r_i^(1-lam) f_a f_b,
// with k the last node r_k <= R: the multipole kernel factorises into a power
// of r times a power of R on either side of R.  k_moments tabulates A and B
// once per basis; per R each integral costs one 16-byte load and two
// multiplies instead of an n_r-term sum.  It is the same quadrature, summed
// in a different association order.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "plan.h"

namespace wpccc {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Partial moments, one thread per Frow entry d = (a, b, lambda); phiT is [n_r+1][n_f].
//   tab[k][d].x = A_k     = sum_{i=1..k}      w_i r_i^(2+lam) f_a(r_i) f_b(r_i)
//   tab[k][d].y = B_(k+1) = sum_{i=k+1..n_r}  w_i r_i^(1-lam) f_a(r_i) f_b(r_i)
__global__ void k_moments(const double* __restrict__ r, const double* __restrict__ w,
                          const double* __restrict__ phiT, const int* __restrict__ da,
                          const int* __restrict__ db, const int* __restrict__ dl, int n_r, int n_f,
                          int n_frow, double2* __restrict__ tab) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n_frow) return;
    const int a = da[d], b = db[d], lam = dl[d];
    double A = 0.0;
    tab[d].x = 0.0;
    for (int i = 1; i <= n_r; ++i) {
        const double ri = r[i];
        double p = ri * ri;
        for (int q = 0; q < lam; ++q) p *= ri;
        A += w[i] * p * phiT[(size_t)i * n_f + a] * phiT[(size_t)i * n_f + b];
        tab[(size_t)i * n_frow + d].x = A;
    }
    double B = 0.0;
    tab[(size_t)n_r * n_frow + d].y = 0.0;
    for (int i = n_r; i >= 1; --i) {
        const double ri = r[i];
        double p;  // r^(1 - lam)
        if (lam == 0) {
            p = ri;
        } else {
            double q = 1.0;
            for (int s = 1; s < lam; ++s) q *= ri;
            p = 1.0 / q;
        }
        B += w[i] * p * phiT[(size_t)i * n_f + a] * phiT[(size_t)i * n_f + b];
        tab[(size_t)(i - 1) * n_frow + d].y = B;
    }
}

// Column mu of Pbar_l^mu = sqrt((l-mu)!/(l+mu)!) P_l^mu(x) (Condon-Shortley
// phase) for l = mu..lam_max, written to pb[pb_index(l, mu)].
__device__ void legendre_column(int lam_max, int mu, double x, double* pb) {
    const double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int i = 1; i <= mu; ++i) pmm *= -sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
    pb[pb_index(mu, mu)] = pmm;
    if (mu + 1 > lam_max) return;
    double p0 = pmm;
    double p1 = sqrt(2.0 * mu + 1.0) * x * pmm;
    pb[pb_index(mu + 1, mu)] = p1;
    for (int l = mu + 1; l < lam_max; ++l) {
        const double p2 = ((2.0 * l + 1.0) * x * p1 - sqrt((double)(l + mu) * (l - mu)) * p0) /
                          sqrt((double)(l + 1 + mu) * (l + 1 - mu));
        pb[pb_index(l + 1, mu)] = p2;
        p0 = p1;
        p1 = p2;
    }
}

// dPbar_l^mu/dx for l = mu..lam_max into pb[pb_index(l, mu)], from
// (x^2 - 1) dPbar_l^mu/dx = l x Pbar_l^mu - sqrt((l+mu)(l-mu)) Pbar_(l-1)^mu, |x| < 1.
__device__ void legendre_column_dx(int lam_max, int mu, double x, double* pb) {
    const double s = sqrt(fmax(0.0, 1.0 - x * x));
    const double den = x * x - 1.0;
    double pmm = 1.0;
    for (int i = 1; i <= mu; ++i) pmm *= -sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
    pb[pb_index(mu, mu)] = mu * x * pmm / den;
    if (mu + 1 > lam_max) return;
    double p0 = pmm;
    double p1 = sqrt(2.0 * mu + 1.0) * x * pmm;
    pb[pb_index(mu + 1, mu)] = ((mu + 1) * x * p1 - sqrt((double)(2 * mu + 1)) * p0) / den;
    for (int l = mu + 1; l < lam_max; ++l) {
        const double p2 = ((2.0 * l + 1.0) * x * p1 - sqrt((double)(l + mu) * (l - mu)) * p0) /
                          sqrt((double)(l + 1 + mu) * (l + 1 - mu));
        pb[pb_index(l + 1, mu)] = ((l + 1) * x * p2 - sqrt((double)(l + 1 + mu) * (l + 1 - mu)) * p1) / den;
        p0 = p1;
        p1 = p2;
    }
}

// Grid node r_k = r_max (k/n_r)^2, with the same arithmetic as the host grid.
__device__ inline double node_r(int k, double r_max, int n_r) {
    const double x = (double)k / n_r;
    return r_max * x * x;
}

// Last grid node with r_k <= R (nodes recomputed in registers).
__device__ inline int grid_index(double R, double r_max, int n_r) {
    int k = (int)floor(n_r * sqrt(fmin(R / r_max, 1.0)));
    k = max(0, min(k, n_r));
    auto rk = [&](int q) { return node_r(q, r_max, n_r); };
    while (k < n_r && rk(k + 1) <= R) ++k;
    while (k > 0 && rk(k) > R) --k;
    return k;
}

// F at R from the table entry (A_k, B_(k+1)).
__device__ inline double radial_at(double2 ab, double R, int lam) {
    double Rl = 1.0;
    for (int q = 0; q < lam; ++q) Rl *= R;
    return ab.x / (Rl * R) + ab.y * Rl;
}

// The R factors of the scaled FP32 table at node k <= R's interval:
// (r_k/R)^(lam+1) (0 at k = 0) and (R/r_(k+1))^lam (0 at k = n_r), both in
// [0, 1] because r_k <= R < r_(k+1).
__device__ inline void scaled_factors(double R, int k, int lam, double r_max, int n_r, double* fa, double* fb) {
    const double qa = k > 0 ? node_r(k, r_max, n_r) / R : 0.0;
    const double qb = k < n_r ? R / node_r(k + 1, r_max, n_r) : 0.0;
    double a = qa, b = 1.0;
    for (int q = 0; q < lam; ++q) {
        a *= qa;
        b *= qb;
    }
    *fa = a;
    *fb = k < n_r ? b : 0.0;
}

// Scaled single-precision copy of the moment table, one thread per (entry d,
// node k): x = A_k / r_k^(lam+1) (0 at k = 0), y = B_(k+1) r_(k+1)^lam (0 at
// k = n_r).  F(R) = x (r_k/R)^(lam+1) + y (R/r_(k+1))^lam is the same
// quadrature as the FP64 table's; the stored values are of the size of the
// integrals (no powers of r that leave FP32's range), rounded once.
__global__ void k_table_f32(const double2* __restrict__ tab, const int* __restrict__ dl, int n_frow, int n_r,
                            double r_max, float2* __restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (d >= n_frow) return;
    const int lam = dl[d];
    const size_t i = (size_t)k * n_frow + d;
    const double2 ab = tab[i];
    double x = 0.0, y = 0.0;
    if (k > 0) {
        const double rk = node_r(k, r_max, n_r);
        double p = rk;
        for (int q = 0; q < lam; ++q) p *= rk;
        x = ab.x / p;
    }
    if (k < n_r) {
        const double rk1 = node_r(k + 1, r_max, n_r);
        double p = 1.0;
        for (int q = 0; q < lam; ++q) p *= rk1;
        y = ab.y * p;
    }
    out[i] = make_float2((float)x, (float)y);
}

// F on the grid nodes, one thread per (entry d, node k): the quadrature of
// Eq. D2 at R = r_k, r_k^-(lam+1) A_k + r_k^lam B_(k+1) (at r_0 = 0 only the
// lam = 0 term B_1 survives).  The paper's production table (Sec. II).
__global__ void k_table_nodes(const double2* __restrict__ tab, const int* __restrict__ dl, int n_frow, int n_r,
                              double r_max, double* __restrict__ out) {
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (d >= n_frow) return;
    const int lam = dl[d];
    const size_t i = (size_t)k * n_frow + d;
    const double2 ab = tab[i];
    double f;
    if (k == 0) {
        f = lam == 0 ? ab.y : 0.0;
    } else {
        const double rk = node_r(k, r_max, n_r);
        double p = 1.0;
        for (int q = 0; q < lam; ++q) p *= rk;
        f = ab.x / (p * rk) + ab.y * p;
    }
    out[i] = f;
}

// Five-point interpolation of the node table at R (R < r_max): the stencil of
// the node j nearest to R in x = sqrt(r/r_max) (uniform in x), nodes j-2..j+2
// clamped to the grid, with the Lagrange weights in r.  Returns the first node.
__device__ inline int interp_stencil(double R, double r_max, int n_r, double* w) {
    int j = (int)rint(n_r * sqrt(R / r_max));
    j = min(max(j, 2), n_r - 2) - 2;
    double x[5];
    for (int i = 0; i < 5; ++i) x[i] = node_r(j + i, r_max, n_r);
    for (int i = 0; i < 5; ++i) {
        double p = 1.0;
        for (int k = 0; k < 5; ++k)
            if (k != i) p *= (R - x[k]) / (x[i] - x[k]);
        w[i] = p;
    }
    return j;
}

// F of entry d (multipole lam) from the node table: the stencil sum (kidx >= 0,
// weights rp[0..4]) or the multipole form beyond the grid, F(r_max) (r_max/R)^(lam+1)
// (kidx = -1, rp[lam] = (r_max/R)^(lam+1)).
__device__ inline double interp_value(const double* ftab, int n_frow, int n_r, int kidx, const double* rp, size_t d,
                                      int lam) {
    if (kidx < 0) return ftab[(size_t)n_r * n_frow + d] * rp[lam];
    double f = 0.0;
    for (int i = 0; i < 5; ++i) f += rp[i] * ftab[(size_t)(kidx + i) * n_frow + d];
    return f;
}

__device__ inline double2 phase(double eps, double z, double v) {
    double sn, cs;
    sincos(eps * z / v, &sn, &cs);
    return make_double2(cs, sn);
}

// Per (path, z-point): grid node of R, powers of R, Pbar table and phases per
// radial function.  grid: x = point, y = path; one wave per block.
__global__ __launch_bounds__(64) void k_prologue(PrologueArgs a) {
    const Meta& m = *a.meta;
    const int j = a.traj0 + blockIdx.y;
    const int p = blockIdx.x;
    const double z = a.zdev ? a.zdev[(size_t)(*a.chunk) * kChunkPoints + p] : a.z[p];
    const double b = a.tb.bvec[j], v = a.tb.vvec[j];
    const double R = sqrt(b * b + z * z);
    const size_t jp = (size_t)j * a.pt.n_pts + p;
    const int t = threadIdx.x;
    const int k = grid_index(R, m.r_max, m.n_r);
    if (a.tb.ftab) {
        // interpolated F: stencil and weights, or the multipole factors beyond the grid
        if (R < m.r_max) {
            if (t == 0) {
                double w[5];
                a.pt.kidx[jp] = interp_stencil(R, m.r_max, m.n_r, w);
                for (int i = 0; i < 5; ++i) a.pt.rpow[jp * kRpow + i] = w[i];
            }
        } else {
            if (t == 0) a.pt.kidx[jp] = -1;
            if (t <= m.lam_max) {
                const double q = m.r_max / R;
                double f = q;
                for (int i = 0; i < t; ++i) f *= q;
                a.pt.rpow[jp * kRpow + t] = f;
            }
        }
    } else if (t == 0) {
        a.pt.kidx[jp] = k;
    }
    if (t <= m.lam_max) {
        if (a.tb.ftab) {
            // factors written above
        } else if (a.tb.tab32) {
            scaled_factors(R, k, t, m.r_max, m.n_r, &a.pt.rpow[jp * kRpow + 2 * t], &a.pt.rpow[jp * kRpow + 2 * t + 1]);
        } else {
            double Rl = 1.0;
            for (int q = 0; q < t; ++q) Rl *= R;
            a.pt.rpow[jp * kRpow + 2 * t] = 1.0 / (Rl * R);
            a.pt.rpow[jp * kRpow + 2 * t + 1] = Rl;
        }
        legendre_column(m.lam_max, t, z / R, a.pt.pbar + jp * kMaxPb);
    }
    for (int f = t; f < m.n_f; f += blockDim.x) a.pt.ph[jp * m.n_f + f] = phase(a.tb.rad_eps[f], z, v);
}

// table entries per thread held in registers by a stage workgroup of `rows`
// rows (about 1.5 per row and thread; the rest is loaded where it is used)
constexpr int fbatch(int rows) { return rows >= 8 ? 12 : (rows * 3 + 1) / 2; }
constexpr int kXBatch = 4;   // amplitudes per thread held in registers
constexpr int kGBatch = 4;   // angular coefficients per thread held in registers

// RK4 combinations (Algorithm 1) of stage `stage` with slope K and step h:
// the next stage input (stages 1-3) and the new accumulator (stages 1-3) or
// the new amplitude (stage 4).
__device__ inline double2 rk4_next_input(int stage, double2 x0, double2 K, double h) {
    const double c = (stage == 3) ? h : 0.5 * h;
    return make_double2(x0.x + c * K.x, x0.y + c * K.y);
}
__device__ inline double2 rk4_accumulate(int stage, double2 x0, double2 xa, double2 K, double h) {
    if (stage == 1) return make_double2(x0.x + h / 6.0 * K.x, x0.y + h / 6.0 * K.y);
    if (stage == 4) return make_double2(xa.x + h / 6.0 * K.x, xa.y + h / 6.0 * K.y);
    return make_double2(xa.x + h / 3.0 * K.x, xa.y + h / 3.0 * K.y);
}

// The RK4 combination of stage a.stage for output oi with slope K and step h.
__device__ inline void rk4_update(const StageArgs& a, size_t oi, double2 K, double2 x0, double2 xa, double h) {
    if (a.stage < 4) {
        a.u_out[oi] = rk4_next_input(a.stage, x0, K, h);
        a.Xacc[oi] = rk4_accumulate(a.stage, x0, xa, K, h);
    } else {
        const double2 xn = rk4_accumulate(4, x0, xa, K, h);
        if (!isfinite(xn.x) || !isfinite(xn.y)) atomicOr(a.flag, 1);
        (a.Xout ? a.Xout : a.X)[oi] = xn;
    }
}

// phase 2 of a stage: W[r][g] = sum_n F_l'[r][e0(g) + n] x'[xoff(g) + n]
// for the workgroup's rows (LDS in, LDS out).  Each work item is one column g
// and half of the rows (ROWS / 2 accumulators), so that every x' load serves
// ROWS / 2 products; lanes of a wave take consecutive g (the F columns of one
// (l, lambda) block are read as a broadcast).
template <int ROWS>
__device__ inline void stage_phase2(const double* Fs, const double2* xs, const int2* gis, double2* Ws, int nrows,
                                    int gcols, int nV) {
    constexpr int RB = (ROWS + 1) / 2;
    const int B = blockDim.x, tid = threadIdx.x;
    for (int it = tid; it < 2 * gcols; it += B) {
        const int half = it >= gcols ? 1 : 0;
        const int g = it - half * gcols;
        const int r0 = half * RB;
        if (r0 >= nrows) continue;
        const int2 info = gis[g];
        const int e0 = info.x & 0xffff, nl = info.x >> 16;
        const double* f = Fs + r0 * nV + e0;
        const double2* x = xs + info.y;
        double re[RB], im[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) re[k] = im[k] = 0.0;
#pragma unroll 2
        for (int n = 0; n < nl; ++n) {
            const double2 y = x[n];
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                // rows r0 + k >= nrows read rows of F that this stage did not
                // fill (inside the ROWS-row buffer); their sums are dropped
                const double fk = f[k * nV + n];
                re[k] += fk * y.x;
                im[k] += fk * y.y;
            }
        }
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (r0 + k < nrows) Ws[(r0 + k) * gcols + g] = make_double2(re[k], im[k]);
    }
}

// phase 3 of a stage: y[r][q'] = sum_g G_l'[q'][g] W[r][g] for output o =
// (r, q') (o < n_out), summed by the S lanes s = 0..S-1 of the output; every
// lane of the wave takes part in the reduction and returns the output's sum.
__device__ inline double2 stage_phase3(const double* Gs, const double2* Ws, int o, int s, int S, int n_out, int nmp,
                                       int gcols) {
    double re = 0.0, im = 0.0;
    if (o < n_out) {
        const int r = o / nmp, qp = o - r * nmp;
        const double* g = Gs + qp * gcols;
        const double2* w = Ws + r * gcols;
        double re1 = 0.0, im1 = 0.0;
        int c = s;
        for (; c + S < gcols; c += 2 * S) {
            const double g0 = g[c], g1 = g[c + S];
            const double2 w0 = w[c], w1 = w[c + S];
            re += g0 * w0.x;
            im += g0 * w0.y;
            re1 += g1 * w1.x;
            im1 += g1 * w1.y;
        }
        if (c < gcols) {
            re += g[c] * w[c].x;
            im += g[c] * w[c].y;
        }
        re += re1;
        im += im1;
    }
    for (int off = S >> 1; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
    }
    return make_double2(re, im);
}

// phase 3 of the large-basis form: as stage_phase3, with the angular factor
// G_l'[q'][g] = c(g) Pbar[p(g)] formed from the coefficient tables (global
// memory, shared by every path and point: L2 hits) instead of staged in LDS.
__device__ inline double2 stage_phase3_global(const double* gc, const int* gp, const double* pbs, const double2* Ws,
                                              int o, int s, int S, int n_out, int nmp, int gcols) {
    double re = 0.0, im = 0.0;
    if (o < n_out) {
        const int r = o / nmp, qp = o - r * nmp;
        const double* c = gc + qp * gcols;
        const int* pp = gp + qp * gcols;
        const double2* w = Ws + r * gcols;
        for (int k = s; k < gcols; k += S) {
            const int p = pp[k];
            if (p >= 0) {
                const double g = c[k] * pbs[p];
                re += g * w[k].x;
                im += g * w[k].y;
            }
        }
    }
    for (int off = S >> 1; off > 0; off >>= 1) {
        re += __shfl_xor(re, off, 64);
        im += __shfl_xor(im, off, 64);
    }
    return make_double2(re, im);
}

// Lanes per output of phase 3: the largest power of two S <= 64 with
// 2 n_out S <= B (so that every output keeps at least half the lanes busy),
// for the n_out = ROWS x (2 l' + 1) outputs of a full tile of the block.
// Every output has a lane group when n_out <= B (phase3_fits).
__device__ inline int phase3_lanes(int n_out, int B) {
    int S = 1;
    while (S < 64 && n_out * S * 2 <= B) S *= 2;
    return S;
}

// Whether a tile of `rows` rows gives every output of blocks of up to
// nmp_max = 2 l_max + 1 values of m' a lane of the stage workgroup.
__host__ __device__ inline bool phase3_fits(int rows, int nmp_max) { return rows * nmp_max <= kStageThreads; }

// One stage for rows [row0, row0 + nrows) of the l' block, all nmp = 2l'+1 values of m'.
// KIND 0: RK4 stage (k_stage); KIND 1: operator application (k_apply, see
// StageArgs) with the same three phases.
//   phase 0: every independent global load of the stage is issued at once
//            (table entries or cached F, stage input, coefficients) and the
//            per-point tables (R powers, Pbar, phases) go to LDS;
//   phase 1: x' = conj(ph) u, F_l'[rows][:] = A R^-(lam+1) + B R^lam (or the
//            cached F), G_l' = c Pbar  -> LDS
//   phase 2: W[r][g] = sum_n F_l'[r][e0(g) + n] x'_{l(g), q(g), n}
//   phase 3: y[r][q'] = sum_g G_l'[q'][g] W[r][g];  K = -(i/v) Zp ph y; RK4 update.
//   phase 4 (FC with a.fc_next): F of the rows at point a.p_next from the
//            moment-table entries loaded in phase 0 -> a.fc_next.
// F32: the moment table is the scaled FP32 form.  FC: F at the stage's point
// comes from the radial-integral cache a.fc_cur (KIND 0 only).  GG (large
// bases, FC only): G_l' is not staged in LDS; phase 3 forms it from the
// coefficient tables.
template <int KIND, int ROWS, bool F32 = false, bool FC = false, bool GG = false>
__device__ void stage_body(const StageArgs& a, int j, const StageTile& t, char* smem) {
    // moment-table entries: FP64 (A_k, B_(k+1)) or the scaled FP32 form
    using TabT = typename std::conditional<F32, float2, double2>::type;
    const Meta& m = *a.meta;
    const Tables& T = a.tb;
    const int N = m.n_states;
    const int row0 = t.row0, nrows = t.nrows;
    const int nmp = t.nmp;
    const int nlp = t.n_l;
    const int nV = t.nV;
    const int gcols = t.gcols;
    const int B = blockDim.x;
    const int tid = threadIdx.x;
    const size_t jp = (size_t)j * a.pt.n_pts + a.p;

    double2* xs = reinterpret_cast<double2*>(smem);                       // [n_xs] (xs_off, xs_stride)
    double2* Ws = xs + m.n_xs;                                             // [rows][gcols]
    double2* phs = Ws + ROWS * gcols;                                      // [n_f]
    double* Fs = reinterpret_cast<double*>(phs + m.n_f);                  // [rows][nV]
    double* Gs = Fs + ROWS * nV;                                           // [nmp][gcols] (not with GG)
    double* rps = GG ? Gs : Gs + nmp * gcols;                              // [kRpow]
    double* pbs = rps + kRpow;                                             // [kMaxPb]
    int2* gis = reinterpret_cast<int2*>(pbs + kMaxPb);                     // [gcols]

    // phase 0
    // the moment-table rows are read at this stage's point (no cache) or at
    // the cache's next point (FC with fc_next)
    const bool tab_rows = !FC || a.fc_next != nullptr;
    const size_t jt = FC ? (size_t)j * a.pt.n_pts + a.p_next : jp;
    const int k = tab_rows ? a.pt.kidx[jt] : 0;
    const TabT* tab = nullptr;
    if constexpr (F32) tab = T.tab32;
    else tab = T.tab;
    const TabT* row = tab + (size_t)k * m.n_frow + t.frow_off + (size_t)row0 * nV;
    // cached F: FP64, or FP32 for the scaled FP32 table
    using FcT = typename std::conditional<F32, float, double>::type;
    const FcT* frow = FC ? static_cast<const FcT*>(a.fc_cur) + (size_t)j * m.n_frow + t.frow_off + (size_t)row0 * nV
                         : nullptr;
    const int* cl = T.col_lam + t.col_off;
    const int totF = nrows * nV;
    constexpr int FB = fbatch(ROWS);
    TabT tv[FB];
    int lv[FB];
    FcT fv[FC ? FB : 1];
    // Every lane loads (past the end: a clamped, in-bounds index whose value
    // is not used), so that all loads of a batch are issued back to back
    // before the first wait: one memory round trip instead of one per batch.
    auto load_table_rows = [&]() {
        int q = tid % nV;
        const int dq = B % nV;
#pragma unroll
        for (int i = 0; i < FB; ++i) {
            tv[i] = row[min(tid + i * B, totF - 1)];
            lv[i] = cl[q];
            q += dq;
            if (q >= nV) q -= nV;
        }
    };
    if (FC) {
        // the next point's table rows are loaded after phase 1, so that they
        // arrive during phases 2 and 3 instead of delaying the first wait
#pragma unroll
        for (int i = 0; i < (FC ? FB : 0); ++i) fv[i] = frow[min(tid + i * B, totF - 1)];
    } else {
        load_table_rows();
    }
    // stage input (KIND 1: v = cu1 u_in + cu2 u_in2)
    const double2* u = a.u_in + (size_t)j * a.n_pad;
    const double2* u2 = (KIND == 1 && a.u_in2) ? a.u_in2 + (size_t)j * a.n_pad : nullptr;
    auto load_u = [&](int idx) -> double2 {
        if (KIND == 0) return u[idx];
        const double2 x = u[idx];
        double2 r = make_double2(a.cu1 * x.x, a.cu1 * x.y);
        if (u2) {
            const double2 y = u2[idx];
            r.x += a.cu2 * y.x;
            r.y += a.cu2 * y.y;
        }
        return r;
    };
    double2 uv[kXBatch];
    int sr[kXBatch], sx[kXBatch];  // radial index and LDS position of each amplitude
#pragma unroll
    for (int i = 0; i < kXBatch; ++i) {
        const int idx = min(tid + i * B, N - 1);
        uv[i] = load_u(idx);
        sr[i] = T.st_rad[idx];
        sx[i] = T.st_xs[idx];
    }
    const double* gc = T.gcoef + t.g_off;
    const int* gp = T.gpb + t.g_off;
    const int totG = nmp * gcols;
    double gcv[kGBatch];
    int gpv[kGBatch];
#pragma unroll
    for (int i = 0; i < kGBatch; ++i) {
        const int idx = min(tid + i * B, totG - 1);
        gcv[i] = GG ? 0.0 : gc[idx];
        gpv[i] = GG ? -1 : gp[idx];
    }
    // output-side values, prefetched by the thread that writes output o.
    // The lanes per output follow from the tiling's ROWS, not from this
    // tile's rows, so that an output sums its columns in the same order in
    // every split of its block (even or greedy tiles, the persistent kernel)
    const int n_out = nrows * nmp;
    const int S = phase3_lanes(ROWS * nmp, B);
    const int o = tid / S, s = tid - o * S;
    const bool writer = (o < n_out) && (s == 0);
    const double v = T.vvec[j];
    size_t oi = 0;
    int rad_o = 0;
    double2 x0 = make_double2(0.0, 0.0), xa = make_double2(0.0, 0.0);
    if (writer) {
        const int r = o / nmp, qp = o - r * nmp;
        oi = (size_t)j * a.n_pad + t.state_off + qp * nlp + row0 + r;
        rad_o = t.rad_off + row0 + r;
        if (KIND == 0) {
            if (a.stage < 4) x0 = a.X[oi];
            if (a.stage > 1) xa = a.Xacc[oi];
        } else {
            // x0 = sum of the added vectors, xa = d = cd1 dv + cd2 dv2
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (a.w[k]) {
                    const double2 t = a.w[k][oi];
                    x0.x += t.x;
                    x0.y += t.y;
                }
            if (a.dv) {
                const double2 t = a.dv[oi];
                xa = make_double2(a.cd1 * t.x, a.cd1 * t.y);
                if (a.dv2) {
                    const double2 t2 = a.dv2[oi];
                    xa.x += a.cd2 * t2.x;
                    xa.y += a.cd2 * t2.y;
                }
            }
        }
    }
    const int deriv = (KIND == 1) ? a.deriv : 0;
    const double bj = T.bvec[j];
    const double Rz = sqrt(bj * bj + a.z * a.z);
    // the point's tables and the column descriptors, one entry per thread
    // (larger tables: the rest is loaded below)
    const int n_rp = 2 * (m.lam_max + 1), n_pb = (m.lam_max + 1) * (m.lam_max + 2) / 2;
    const int2 gv = T.gcol_info[t.gcol_off + min(tid, gcols - 1)];
    const double rpv = tab_rows ? a.pt.rpow[jt * kRpow + min(tid, n_rp - 1)] : 0.0;
    const double pbv = a.pt.pbar[jp * kMaxPb + min(tid, n_pb - 1)];
    const double2 phv = a.pt.ph[jp * m.n_f + min(tid, m.n_f - 1)];
    // every load above is issued before any of their values is used
    __builtin_amdgcn_sched_barrier(0);
    if (deriv == 1) {
        // d/dR of R^-(lam+1) and R^lam
        if (tid <= m.lam_max) {
            double Rl = 1.0;
            for (int q = 0; q < tid; ++q) Rl *= Rz;
            rps[2 * tid] = -(tid + 1.0) / (Rl * Rz * Rz);
            rps[2 * tid + 1] = tid > 0 ? tid * Rl / Rz : 0.0;
        }
    } else if (tid < n_rp) {
        rps[tid] = rpv;
    }
    if (tid < gcols) gis[tid] = gv;
    for (int i = tid + B; i < gcols; i += B) gis[i] = T.gcol_info[t.gcol_off + i];
    if (deriv == 2) {
        if (tid <= m.lam_max) legendre_column_dx(m.lam_max, tid, a.z / Rz, pbs);
    } else {
        if (tid < n_pb) pbs[tid] = pbv;
        for (int i = tid + B; i < n_pb; i += B) pbs[i] = a.pt.pbar[jp * kMaxPb + i];
    }
    if (tid < m.n_f) phs[tid] = phv;
    for (int i = tid + B; i < m.n_f; i += B) phs[i] = a.pt.ph[jp * m.n_f + i];
    __syncthreads();

    // phase 1
#pragma unroll
    for (int i = 0; i < kXBatch; ++i) {
        const int idx = tid + i * B;
        if (idx < N) {
            const double2 ph = phs[sr[i]], x = uv[i];
            xs[sx[i]] = make_double2(ph.x * x.x + ph.y * x.y, ph.x * x.y - ph.y * x.x);
        }
    }
    for (int idx = tid + kXBatch * B; idx < N; idx += B) {
        const double2 ph = phs[T.st_rad[idx]], x = load_u(idx);
        xs[T.st_xs[idx]] = make_double2(ph.x * x.x + ph.y * x.y, ph.x * x.y - ph.y * x.x);
    }
    if (FC) {
#pragma unroll
        for (int i = 0; i < (FC ? FB : 0); ++i) {
            const int idx = tid + i * B;
            if (idx < totF) Fs[idx] = (double)fv[i];
        }
        for (int idx = tid + FB * B; idx < totF; idx += B) Fs[idx] = (double)frow[idx];
    } else {
#pragma unroll
        for (int i = 0; i < FB; ++i) {
            const int idx = tid + i * B;
            if (idx < totF) Fs[idx] = (double)tv[i].x * rps[2 * lv[i]] + (double)tv[i].y * rps[2 * lv[i] + 1];
        }
        for (int idx = tid + FB * B; idx < totF; idx += B) {
            const TabT t0 = row[idx];
            const int l0 = cl[idx % nV];
            Fs[idx] = (double)t0.x * rps[2 * l0] + (double)t0.y * rps[2 * l0 + 1];
        }
    }
    if (!GG) {
#pragma unroll
        for (int i = 0; i < kGBatch; ++i) {
            const int idx = tid + i * B;
            if (idx < totG) Gs[idx] = gpv[i] >= 0 ? gcv[i] * pbs[gpv[i]] : 0.0;
        }
        for (int idx = tid + kGBatch * B; idx < totG; idx += B) {
            const int p = gp[idx];
            Gs[idx] = p >= 0 ? gc[idx] * pbs[p] : 0.0;
        }
    }
    __syncthreads();

    if (FC && tab_rows) load_table_rows();
    stage_phase2<ROWS>(Fs, xs, gis, Ws, nrows, gcols, nV);
    __syncthreads();
    const double2 y = GG ? stage_phase3_global(gc, gp, pbs, Ws, o, s, S, n_out, nmp, gcols)
                         : stage_phase3(Gs, Ws, o, s, S, n_out, nmp, gcols);
    double gval = 0.0, gma = 0.0, gmc = 0.0;
    if (writer) {
        const double2 py = cmul(phs[rad_o], y);
        const double sc = a.Zp / v;
        double2 K = make_double2(sc * py.y, -sc * py.x);  // -(i/v) Zp ph y
        const double h = a.h;
        if (KIND == 1) {
            if (deriv) {
                const double f = deriv == 1 ? bj / Rz : -a.z * bj / (Rz * Rz * Rz);
                K = make_double2(f * K.x, f * K.y);
            }
            if (a.out) a.out[oi] = make_double2(a.alpha * K.x + x0.x, a.alpha * K.y + x0.y);
            gval = 2.0 * a.gamma * (xa.x * K.x + xa.y * K.y);  // 2 gamma Re(conj(d) K)
            if (a.model) {
                // (dDeltaV/dtheta)_{n' n} x'_n over the radial block of (l', q'):
                // dM/dtheta v = -(i/v) ph (dDeltaV/dtheta) conj(ph) v and x' = conj(ph) v
                const int r = o / nmp, qp = o - r * nmp;
                const double* fa = a.va + t.vo + (size_t)(row0 + r) * nlp;
                const double* fc = a.vc + t.vo + (size_t)(row0 + r) * nlp;
                const double2* xq = xs + t.xs_off + qp * t.xs_stride;
                double2 ca = make_double2(0.0, 0.0), cc = make_double2(0.0, 0.0);
                for (int n = 0; n < nlp; ++n) {
                    const double2 x = xq[n];
                    ca.x += fa[n] * x.x;
                    ca.y += fa[n] * x.y;
                    cc.x += fc[n] * x.x;
                    cc.y += fc[n] * x.y;
                }
                const double2 p = phs[rad_o];
                const double2 t = make_double2(xa.x * p.x + xa.y * p.y, xa.x * p.y - xa.y * p.x);  // conj(d) p
                // 2 gamma Re(-(i/v) t c) = 2 gamma Im(t c) / v
                gma = 2.0 * a.gamma * (t.x * ca.y + t.y * ca.x) / v;
                gmc = 2.0 * a.gamma * (t.x * cc.y + t.y * cc.x) / v;
            }
        } else {
            // graph replays read the step length from device memory
            const double hh = a.hdev ? a.hdev[(size_t)(*a.chunk) * kChunkSteps + a.hidx] : h;
            rk4_update(a, oi, K, x0, xa, hh);
        }
    }
    if (FC && a.fc_next) {
        // phase 4: the cache's next point (rps holds its R factors)
        FcT* fout = static_cast<FcT*>(a.fc_next) + (size_t)j * m.n_frow + t.frow_off + (size_t)row0 * nV;
#pragma unroll
        for (int i = 0; i < FB; ++i) {
            const int idx = tid + i * B;
            if (idx < totF) fout[idx] = (FcT)((double)tv[i].x * rps[2 * lv[i]] + (double)tv[i].y * rps[2 * lv[i] + 1]);
        }
        for (int idx = tid + FB * B; idx < totF; idx += B) {
            const TabT t0 = row[idx];
            const int l0 = cl[idx % nV];
            fout[idx] = (FcT)((double)t0.x * rps[2 * l0] + (double)t0.y * rps[2 * l0 + 1]);
        }
    }
    if (KIND == 1 && a.grad) {
        // this workgroup's shares, accumulated over the launches in its own
        // slots and summed in a fixed order by k_grad_sum
        __shared__ double red[3][kStageThreads / 64];
        for (int off = 32; off > 0; off >>= 1) {
            gval += __shfl_xor(gval, off, 64);
            gma += __shfl_xor(gma, off, 64);
            gmc += __shfl_xor(gmc, off, 64);
        }
        if ((tid & 63) == 0) {
            red[0][tid >> 6] = gval;
            red[1][tid >> 6] = gma;
            red[2][tid >> 6] = gmc;
        }
        __syncthreads();
        if (tid == 0) {
            double sb = 0.0, sa = 0.0, sc = 0.0;
            for (int w = 0; w < B / 64; ++w) {
                sb += red[0][w];
                sa += red[1][w];
                sc += red[2][w];
            }
            double* g = a.grad + (size_t)j * kGradSlots * gridDim.x + blockIdx.x;
            g[a.gslot * gridDim.x] += sb;
            if (a.model) {
                g[2 * gridDim.x] += sa;
                g[3 * gridDim.x] += sc;
            }
        }
    }
}

// k_apply's grid: x = row tile of a path (a.tiles, l' order), y = path.
template <int KIND, int ROWS, bool GG = false>
__device__ void stage_entry(const StageArgs& a, char* smem) {
    const StageTile t = a.tiles[blockIdx.x];
    if (t.nrows <= 0) return;
    stage_body<KIND, ROWS, false, false, GG>(a, a.traj0 + blockIdx.y, t, smem);
}

__device__ inline int chunks_of(const Meta& m, int rows) {
    int n = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) n += (m.n_l[lp] + rows - 1) / rows;
    return n;
}

// Work item of workgroup bx in a one-dimensional grid of 8 x ceil(items / 8)
// workgroups over items = paths x row chunks (path-major): consecutive
// workgroup ids go to the eight XCDs in turn and the items of XCD x are the
// x-th eighth of the list, so the workgroups of a path share an XCD (and its
// L2, which then serves the path's stage input to all of them).  Returns
// false for the padding workgroups.
template <int ROWS>
__device__ inline bool xcd_item(const Meta& m, int n_paths, int bx, int* jl, int* lp, int* row0, int* nrows) {
    const int nwg = chunks_of(m, ROWS);
    const int total = n_paths * nwg;
    const int per = (total + 7) / 8;
    const int W = (bx % 8) * per + bx / 8;
    if (W >= total) return false;
    *jl = W / nwg;
    int ci = W - *jl * nwg, l = 0;
    for (; l < m.l_max; ++l) {
        const int nc = (m.n_l[l] + ROWS - 1) / ROWS;
        if (ci < nc) break;
        ci -= nc;
    }
    *lp = l;
    *row0 = ci * ROWS;
    *nrows = min(ROWS, m.n_l[l] - *row0);
    return *nrows > 0;
}

// One RK4 stage for a.n_paths paths from a.traj0 (grid of xcd_item).  Small
// row tiles ask for registers that leave room for four workgroups per CU
// (their LDS does), larger ones for three.
template <int ROWS, bool F32, bool FC, bool GG = false>
__global__ __launch_bounds__(kStageThreads, ROWS <= 4 ? 4 : 3) void k_stage(StageArgs a) {
    extern __shared__ double2 smem2[];
    // work item W of the path-major list of a.n_paths x a.nwg row tiles, in
    // the XCD order of xcd_item; the tile (one 64-byte load) holds the
    // per-l' offsets, so no loop over the basis blocks precedes the loads
    const int total = a.n_paths * a.nwg;
    const int per = (total + 7) / 8;
    const int W = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (W >= total) return;
    const int jl = W / a.nwg;
    const StageTile t = a.tiles[W - jl * a.nwg];
    stage_body<0, ROWS, F32, FC, GG>(a, a.traj0 + jl, t, reinterpret_cast<char*>(smem2));
}

// F of Eq. D2 at point slot p for every entry of the row layout and every path
// of the launch (grid: entries / 256 x paths), with the arithmetic of the
// stage kernels' phase 1 / phase 4.
template <bool F32>
__global__ __launch_bounds__(256) void k_fpoint(const Meta* __restrict__ mp_, Tables T, PointArrays pt, int p,
                                                int traj0, void* __restrict__ fc_) {
    const Meta& m = *mp_;
    const int d = blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= m.n_frow) return;
    const int j = traj0 + blockIdx.y;
    const size_t jp = (size_t)j * pt.n_pts + p;
    int lp = 0;
    while (lp < m.l_max && d >= m.frow_off[lp + 1]) ++lp;
    const int lam = T.col_lam[m.col_off[lp] + (d - m.frow_off[lp]) % m.nV[lp]];
    const double* rp = pt.rpow + jp * kRpow;
    if (T.ftab) {
        static_cast<double*>(fc_)[(size_t)j * m.n_frow + d] =
            interp_value(T.ftab, m.n_frow, m.n_r, pt.kidx[jp], rp, d, lam);
        return;
    }
    const size_t i = (size_t)pt.kidx[jp] * m.n_frow + d;
    if constexpr (F32) {
        const float2 t0 = T.tab32[i];
        static_cast<float*>(fc_)[(size_t)j * m.n_frow + d] =
            (float)((double)t0.x * rp[2 * lam] + (double)t0.y * rp[2 * lam + 1]);
    } else {
        const double2 t0 = T.tab[i];
        static_cast<double*>(fc_)[(size_t)j * m.n_frow + d] = t0.x * rp[2 * lam] + t0.y * rp[2 * lam + 1];
    }
}

constexpr int kBarrierSpin = 1 << 22;  // polls (0.2 s or more) before a barrier gives up

// Barrier of the workgroups of one path, in two halves so that loads that do
// not depend on the other workgroups can be issued in between.
// path_arrive: every wave waits until its own memory operations are done
// (stores in the L2), then thread 0 arrives with an agent-scope release
// (which writes the L2 back for the other XCDs).
// path_wait: thread 0 polls the counter with relaxed loads until `target`
// workgroups have arrived and acquires at agent scope once; the workgroup
// barrier orders the other waves' reads after that acquire.  A wait longer
// than kBarrierSpin polls latches bit 2 of *flag and returns false, so every
// workgroup still ends.
__device__ inline void path_arrive(int* cnt) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ bool path_wait(int* cnt, int target, int* flag) {
    __shared__ int ok;
    if (threadIdx.x == 0) {
        ok = 1;
        int it = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++it > kBarrierSpin) {
                atomicOr(flag, 2);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return ok != 0;
}

// table entries per thread k_chunk prefetches into registers (14 covers
// 12 rows of 300 columns; smaller tiles need fewer)
constexpr int fpre(int rows) { return rows >= 10 ? 14 : fbatch(rows) + 1; }

// Per-thread state of a k_chunk workgroup, kept in registers across stages.
template <int FP>
struct ChunkRegs {
    double2 tv[FP];     // the next new point's table entries (this thread's share) ...
    double rp, pb;         // ... its R power, Pbar entry
    double2 ph;            // ... and phase (radial function tid)
    double gcv[kGBatch];   // angular coefficients of l' (constant)
    int gpv[kGBatch];
    int sv[kXBatch];       // radial index | LDS position << 16 of the amplitudes this thread converts (constant)
    double2 x0, xa;        // writer: amplitude at the start of the step, RK4 accumulator
};

// Loads of point p's data for the workgroup's rows into registers; they are
// consumed by the next stage at a new point, after the path barrier.
template <int FP>
__device__ inline void chunk_prefetch(const StageArgs& a, int j, int lp, int row0, int nrows, int p, ChunkRegs<FP>& r) {
    const Meta& m = *a.meta;
    const int B = blockDim.x, tid = threadIdx.x, nV = m.nV[lp];
    const size_t jp = (size_t)j * a.pt.n_pts + p;
    const int k = a.pt.kidx[jp];
    const double2* row = a.tb.tab + (size_t)k * m.n_frow + m.frow_off[lp] + (size_t)row0 * nV;
    const int totF = nrows * nV;
#pragma unroll
    for (int i = 0; i < FP; ++i) {
        const int idx = tid + i * B;
        if (idx < totF) r.tv[i] = row[idx];
    }
    if (tid < 2 * (m.lam_max + 1)) r.rp = a.pt.rpow[jp * kRpow + tid];
    if (tid < (m.lam_max + 1) * (m.lam_max + 2) / 2) r.pb = a.pt.pbar[jp * kMaxPb + tid];
    if (tid < m.n_f) r.ph = a.pt.ph[jp * m.n_f + tid];
}

// One RK4 stage of k_chunk for rows [row0, row0 + nrows) of l': the
// arithmetic of stage_body (KIND 0), with the point's data taken from the
// prefetch registers (fresh) or left in LDS by the previous stage (!fresh),
// and the writer's X and accumulator kept in registers.
template <int ROWS>
__device__ void chunk_stage(const StageArgs& a, int j, int lp, int row0, int nrows, char* smem, bool fresh,
                            ChunkRegs<fpre(ROWS)>& r) {
    constexpr int FP = fpre(ROWS);
    const Meta& m = *a.meta;
    const Tables& T = a.tb;
    const int N = m.n_states;
    const int nmp = 2 * lp + 1;
    const int nlp = m.n_l[lp];
    const int nV = m.nV[lp];
    const int gcols = m.gcols[lp];
    const int B = blockDim.x;
    const int tid = threadIdx.x;
    const size_t jp = (size_t)j * a.pt.n_pts + a.p;

    double2* xs = reinterpret_cast<double2*>(smem);
    double2* Ws = xs + m.n_xs;
    double2* phs = Ws + ROWS * gcols;
    double* Fs = reinterpret_cast<double*>(phs + m.n_f);
    double* Gs = Fs + ROWS * nV;
    double* rps = Gs + nmp * gcols;
    double* pbs = rps + kRpow;
    int2* gis = reinterpret_cast<int2*>(pbs + kMaxPb);
    const int* cls = reinterpret_cast<const int*>(gis + gcols);  // multipole order of each F column

    const double2* u = a.u_in + (size_t)j * a.n_pad;
    double2 uv[kXBatch];
#pragma unroll
    for (int i = 0; i < kXBatch; ++i) {
        const int idx = tid + i * B;
        if (idx < N) uv[i] = u[idx];
    }
    if (fresh) {
        if (tid < 2 * (m.lam_max + 1)) rps[tid] = r.rp;
        if (tid < (m.lam_max + 1) * (m.lam_max + 2) / 2) pbs[tid] = r.pb;
        if (tid < m.n_f) phs[tid] = r.ph;
        for (int i = tid + B; i < m.n_f; i += B) phs[i] = a.pt.ph[jp * m.n_f + i];
    }
    __syncthreads();

#pragma unroll
    for (int i = 0; i < kXBatch; ++i) {
        const int idx = tid + i * B;
        if (idx < N) {
            const double2 ph = phs[r.sv[i] & 0xffff], x = uv[i];
            xs[r.sv[i] >> 16] = make_double2(ph.x * x.x + ph.y * x.y, ph.x * x.y - ph.y * x.x);
        }
    }
    for (int idx = tid + kXBatch * B; idx < N; idx += B) {
        const double2 ph = phs[T.st_rad[idx]], x = u[idx];
        xs[T.st_xs[idx]] = make_double2(ph.x * x.x + ph.y * x.y, ph.x * x.y - ph.y * x.x);
    }
    if (fresh) {
        const int totF = nrows * nV;
#pragma unroll
        for (int i = 0; i < FP; ++i) {
            const int idx = tid + i * B;
            if (idx < totF) {
                const int l0 = cls[idx % nV];
                Fs[idx] = r.tv[i].x * rps[2 * l0] + r.tv[i].y * rps[2 * l0 + 1];
            }
        }
        if (totF > FP * B) {
            const double2* row = T.tab + (size_t)a.pt.kidx[jp] * m.n_frow + m.frow_off[lp] + (size_t)row0 * nV;
            for (int idx = tid + FP * B; idx < totF; idx += B) {
                const double2 t0 = row[idx];
                const int l0 = cls[idx % nV];
                Fs[idx] = t0.x * rps[2 * l0] + t0.y * rps[2 * l0 + 1];
            }
        }
        const int totG = nmp * gcols;
#pragma unroll
        for (int i = 0; i < kGBatch; ++i) {
            const int idx = tid + i * B;
            if (idx < totG) Gs[idx] = r.gpv[i] >= 0 ? r.gcv[i] * pbs[r.gpv[i]] : 0.0;
        }
        const double* gc = T.gcoef + m.g_off[lp];
        const int* gp = T.gpb + m.g_off[lp];
        for (int idx = tid + kGBatch * B; idx < totG; idx += B) {
            const int p = gp[idx];
            Gs[idx] = p >= 0 ? gc[idx] * pbs[p] : 0.0;
        }
    }
    __syncthreads();

    stage_phase2<ROWS>(Fs, xs, gis, Ws, nrows, gcols, nV);
    __syncthreads();
    const int n_out = nrows * nmp;
    const int S = phase3_lanes(ROWS * nmp, B);   // as stage_body
    const int o = tid / S, s = tid - o * S;
    const double2 y = stage_phase3(Gs, Ws, o, s, S, n_out, nmp, gcols);
    if (o < n_out && s == 0) {
        const int rr = o / nmp, qp = o - rr * nmp;
        const size_t oi = (size_t)j * a.n_pad + m.state_off[lp] + qp * nlp + row0 + rr;
        const double2 py = cmul(phs[m.rad_off[lp] + row0 + rr], y);
        const double sc = a.Zp / T.vvec[j];
        const double2 K = make_double2(sc * py.y, -sc * py.x);  // -(i/v) Zp ph y
        if (a.stage < 4) {
            a.u_out[oi] = rk4_next_input(a.stage, r.x0, K, a.h);
            r.xa = rk4_accumulate(a.stage, r.x0, r.xa, K, a.h);
        } else {
            const double2 xn = rk4_accumulate(4, r.x0, r.xa, K, a.h);
            if (!isfinite(xn.x) || !isfinite(xn.y)) atomicOr(a.flag, 1);
            a.X[oi] = xn;
            r.x0 = xn;
        }
    }
}

// All steps of a chunk for every path (see ChunkArgs).  grid: 8 x ceil(items
// / 8) workgroups, items = paths x row chunks; consecutive workgroup ids go to
// the eight XCDs in turn and the items of XCD x are the x-th eighth of the
// path-major list, so the workgroups of a path share an XCD (and its L2).
// Each workgroup keeps the couplings of its rows at the current point in LDS
// and builds them only when the point changes (twice per step: midpoint and
// end point); the loads for the next new point are issued before the path
// barrier that precedes it, so their latency overlaps the wait.
template <int ROWS>
__global__ __launch_bounds__(kStageThreads, 2) void k_chunk(ChunkArgs c) {
    extern __shared__ double2 smem2[];
    char* smem = reinterpret_cast<char*>(smem2);
    const Meta& m = *c.s.meta;
    const Tables& T = c.s.tb;
    const int nwg = chunks_of(m, ROWS);
    int jl, lp, row0, nrows;
    if (!xcd_item<ROWS>(m, c.n_traj, blockIdx.x, &jl, &lp, &row0, &nrows)) return;
    const int j = c.s.traj0 + jl;
    const int B = blockDim.x, tid = threadIdx.x;
    const int N = m.n_states, nmp = 2 * lp + 1, nV = m.nV[lp], gcols = m.gcols[lp];

    // constants of the workgroup's rows
    ChunkRegs<fpre(ROWS)> r;
    {
        const double* gc = T.gcoef + m.g_off[lp];
        const int* gp = T.gpb + m.g_off[lp];
#pragma unroll
        for (int i = 0; i < kGBatch; ++i) {
            const int idx = tid + i * B;
            r.gcv[i] = idx < nmp * gcols ? gc[idx] : 0.0;
            r.gpv[i] = idx < nmp * gcols ? gp[idx] : -1;
        }
#pragma unroll
        for (int i = 0; i < kXBatch; ++i) {
            const int idx = tid + i * B;
            r.sv[i] = idx < N ? (T.st_rad[idx] | (T.st_xs[idx] << 16)) : 0;
        }
        double* Fs = reinterpret_cast<double*>(reinterpret_cast<double2*>(smem) + m.n_xs + ROWS * gcols + m.n_f);
        int2* gis = reinterpret_cast<int2*>(Fs + ROWS * nV + nmp * gcols + kRpow + kMaxPb);
        for (int i = tid; i < gcols; i += B) gis[i] = T.gcol_info[m.gcol_off[lp] + i];
        int* cls = reinterpret_cast<int*>(gis + gcols);
        for (int i = tid; i < nV; i += B) cls[i] = T.col_lam[m.col_off[lp] + i];
        const int n_out = nrows * nmp;
        const int S = phase3_lanes(ROWS * nmp, B);   // as stage_body
        const int o = tid / S;
        r.x0 = r.xa = make_double2(0.0, 0.0);
        if (o < n_out && tid - o * S == 0) {
            const int rr = o / nmp, qp = o - rr * nmp;
            r.x0 = c.s.X[(size_t)j * c.s.n_pad + m.state_off[lp] + qp * m.n_l[lp] + row0 + rr];
        }
    }
    StageArgs a = c.s;
    chunk_prefetch(a, j, lp, row0, nrows, 0, r);
    int target = 0;
    for (int i = 0; i < c.n_steps; ++i) {
        a.h = c.h[i];
        for (int stage = 1; stage <= 4; ++stage) {
            a.stage = stage;
            a.p = stage == 1 ? 2 * i : (stage == 4 ? 2 * i + 2 : 2 * i + 1);
            a.u_in = stage == 1 ? c.s.X : (stage == 3 ? c.Ub : c.Ua);
            a.u_out = stage == 1 ? c.Ua : (stage == 2 ? c.Ub : (stage == 3 ? c.Ua : nullptr));
            // stage 3 repeats stage 2's point (the midpoint) and stage 1 of
            // step i > 0 repeats stage 4's point of step i - 1
            const bool fresh = stage == 2 || stage == 4 || i == 0;
            chunk_stage<ROWS>(a, j, lp, row0, nrows, smem, fresh, r);
            if (i + 1 == c.n_steps && stage == 4) break;
            int* bar = c.bar + (size_t)jl * kBarStride;
            path_arrive(bar);
            // the next stage at a new point: stage 2 (midpoint) or 4 (end point)
            if (stage == 1 || stage == 3) chunk_prefetch(a, j, lp, row0, nrows, 2 * i + (stage == 1 ? 1 : 2), r);
            target += nwg;
            if (!path_wait(bar, target, c.s.flag)) return;
        }
    }
}

// Operator application with the grid of k_stage (see StageArgs), ROWS rows
// per workgroup (kRowsPerBlock, or kApplyRowsLarge where that does not fit
// the LDS); GG: the large-basis form (angular factors formed in phase 3 from
// the coefficient tables, F from the moment table as in every k_apply).
template <int ROWS, bool GG = false>
__global__ __launch_bounds__(kStageThreads) void k_apply(ApplyArgs a) {
    extern __shared__ double2 smem2[];
    stage_entry<1, ROWS, GG>(a.s[blockIdx.z], reinterpret_cast<char*>(smem2));
}

// grad[j] = (dL/da, dL/dc, dL/db): the k_apply shares of path j (slots 2, 3
// and 0 + 1 of gpart[j][kGradSlots][n_part]) summed in a fixed order, so that
// the result does not depend on the order in which workgroups ran.
__global__ __launch_bounds__(64) void k_grad_sum(const double* __restrict__ gpart, int n_part,
                                                 double* __restrict__ grad) {
    const int j = blockIdx.x, t = threadIdx.x;
    if (t >= 3) return;
    const double* g = gpart + (size_t)j * kGradSlots * n_part;
    double s = 0.0;
    if (t < 2) {
        for (int i = 0; i < n_part; ++i) s += g[(2 + t) * n_part + i];
    } else {
        for (int i = 0; i < 2 * n_part; ++i) s += g[i];
    }
    grad[(size_t)j * 3 + t] = s;
}

__global__ void k_chunk_counter(int* chunk, int reset) {
    if (reset) *chunk = 0;
    else *chunk += 1;
}

// tab[k][idx[e]].y += val[e] for every grid node k; grid (entries, nodes)
__global__ void k_table_shift(double2* __restrict__ tab, int n_frow, const int* __restrict__ idx,
                              const double* __restrict__ val, int count) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    tab[(size_t)blockIdx.y * n_frow + idx[e]].y += val[e];
}

// Diagnostic path: Frow, G and phases of one (path, z) into scratch arrays.
// grid: x = [nbF Frow blocks | nbP phase blocks | G blocks].
__global__ __launch_bounds__(256) void k_slot_setup(SetupArgs a) {
    const Meta& m = *a.meta;
    const Tables& T = a.tb;
    const double z = a.z;
    const double b = T.bvec[a.j], v = T.vvec[a.j];
    const double R = sqrt(b * b + z * z);
    const int bx = blockIdx.x;
    if (bx < a.nbF) {
        const int d = bx * blockDim.x + threadIdx.x;
        if (d >= m.n_frow) return;
        int lp = 0;
        while (lp < m.l_max && d >= m.frow_off[lp + 1]) ++lp;
        const int e = (d - m.frow_off[lp]) % m.nV[lp];
        const int k = grid_index(R, m.r_max, m.n_r);
        const int lam = T.col_lam[m.col_off[lp] + e];
        if (T.ftab) {
            double rp[kRpow];
            int kk = -1;
            if (R < m.r_max) {
                kk = interp_stencil(R, m.r_max, m.n_r, rp);
            } else {
                double f = m.r_max / R;
                for (int q = 0; q <= lam; ++q) {
                    rp[q] = f;
                    f *= m.r_max / R;
                }
            }
            a.Frow[d] = interp_value(T.ftab, m.n_frow, m.n_r, kk, rp, d, lam);
        } else if (T.tab32) {
            const float2 ab = T.tab32[(size_t)k * m.n_frow + d];
            double fa, fb;
            scaled_factors(R, k, lam, m.r_max, m.n_r, &fa, &fb);
            a.Frow[d] = (double)ab.x * fa + (double)ab.y * fb;
        } else {
            a.Frow[d] = radial_at(T.tab[(size_t)k * m.n_frow + d], R, lam);
        }
        return;
    }
    if (bx < a.nbF + a.nbP) {
        const int i = (bx - a.nbF) * blockDim.x + threadIdx.x;
        if (i < m.n_states) a.PH[i] = phase(T.eps[i], z, v);
        return;
    }
    __shared__ double pb[kMaxPb];
    if ((int)threadIdx.x <= m.lam_max) legendre_column(m.lam_max, threadIdx.x, z / R, pb);
    __syncthreads();
    const int i = (bx - a.nbF - a.nbP) * blockDim.x + threadIdx.x;
    if (i < m.n_g) {
        const int p = T.gpb[i];
        a.G[i] = p >= 0 ? T.gcoef[i] * pb[p] : 0.0;
    }
}

// Dense D_T (Eq. D1) with phases: H[row][col] = Zp ph_row conj(ph_col) sum_lambda G F.
__global__ void k_couplings_dense(const Meta* __restrict__ mp_, const double* __restrict__ Frow,
                                  const double* __restrict__ G, const double2* __restrict__ PH, double Zp,
                                  double2* __restrict__ H) {
    const Meta& m = *mp_;
    const int N = m.n_states;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (col >= N) return;
    int lp = 0, l = 0;
    while (lp < m.l_max && row >= m.state_off[lp + 1]) ++lp;
    while (l < m.l_max && col >= m.state_off[l + 1]) ++l;
    const int rp = row - m.state_off[lp], rc = col - m.state_off[l];
    const int qp = rp / m.n_l[lp], np = rp - qp * m.n_l[lp];
    const int q = rc / m.n_l[l], n = rc - q * m.n_l[l];
    int e0 = 0, g0 = 0;
    for (int ll = 0; ll < l; ++ll) {
        const int nlam = min(ll, lp) + 1;
        e0 += nlam * m.n_l[ll];
        g0 += nlam * (2 * ll + 1);
    }
    const double* Fr = Frow + m.frow_off[lp] + (size_t)np * m.nV[lp];
    const double* Gr = G + m.g_off[lp] + (size_t)qp * m.gcols[lp];
    double acc = 0.0;
    for (int lam = abs(l - lp); lam <= l + lp; lam += 2) {
        acc += Gr[g0 + q] * Fr[e0 + n];
        e0 += m.n_l[l];
        g0 += 2 * l + 1;
    }
    const double2 pr = PH[row], pc = PH[col];
    const double2 w = make_double2(pr.x * pc.x + pr.y * pc.y, pr.y * pc.x - pr.x * pc.y);  // pr conj(pc)
    H[(size_t)row * N + col] = make_double2(Zp * acc * w.x, Zp * acc * w.y);
}

__global__ void k_probabilities(const double2* __restrict__ X, int n_states, int n_pad,
                                double* __restrict__ P, double* __restrict__ norm) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n_states; i += blockDim.x) {
        const double2 x = X[(size_t)j * n_pad + i];
        const double p = x.x * x.x + x.y * x.y;
        if (P) P[(size_t)j * n_pad + i] = p;
        s += p;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && norm) norm[j] = red[0];
}

}  // namespace

int stage_chunks(const Meta& m, int rows) {
    int n = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) n += (m.n_l[lp] + rows - 1) / rows;
    return n;
}

namespace {
// Rows [r0, r0 + nrows) of block l' of one path (vo: offset of the block's
// model-potential rows).
StageTile make_tile(const Meta& m, int lp, int r0, int nrows, int vo) {
    StageTile t{};
    t.lp = lp;
    t.row0 = r0;
    t.nrows = nrows;
    t.nmp = 2 * lp + 1;
    t.nV = m.nV[lp];
    t.gcols = m.gcols[lp];
    t.frow_off = m.frow_off[lp];
    t.col_off = m.col_off[lp];
    t.g_off = m.g_off[lp];
    t.gcol_off = m.gcol_off[lp];
    t.state_off = m.state_off[lp];
    t.rad_off = m.rad_off[lp];
    t.n_l = m.n_l[lp];
    t.xs_off = m.xs_off[lp];
    t.xs_stride = m.xs_stride[lp];
    t.vo = vo;
    return t;
}
}  // namespace

void stage_tiles(const Meta& m, int rows, std::vector<StageTile>& out) {
    out.clear();
    int vo = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        for (int r0 = 0; r0 < m.n_l[lp]; r0 += rows) out.push_back(make_tile(m, lp, r0, std::min(rows, m.n_l[lp] - r0), vo));
        vo += m.n_l[lp] * m.n_l[lp];
    }
}

void stage_tiles_balanced(const Meta& m, int rows, int n_launch, long long wg_slots, std::vector<StageTile>& out) {
    out.clear();
    int cap[kMaxL + 1];
    long long per_path = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        cap[lp] = rows;
        per_path += (m.n_l[lp] + rows - 1) / rows;
    }
    for (int lp = m.l_max; lp >= 0 && rows > 1; --lp) {
        const int extra = (m.n_l[lp] + rows - 2) / (rows - 1) - (m.n_l[lp] + rows - 1) / rows;
        if ((long long)n_launch * (per_path + extra) <= wg_slots) {
            cap[lp] = rows - 1;
            per_path += extra;
        }
    }
    int vo = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        const int n = m.n_l[lp], nt = (n + cap[lp] - 1) / cap[lp];
        for (int ti = 0, r0 = 0; ti < nt; ++ti) {
            const int nr = n / nt + (ti < n % nt ? 1 : 0);
            out.push_back(make_tile(m, lp, r0, nr, vo));
            r0 += nr;
        }
        vo += n * n;
    }
}

int stage_smem_bytes(const Meta& m, int rows, bool gg) {
    int best = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        const size_t nmp = gg ? 0 : 2 * lp + 1;
        const size_t bytes = m.n_xs * sizeof(double2) + (size_t)rows * m.gcols[lp] * sizeof(double2) +
                             (size_t)m.n_f * sizeof(double2) + (size_t)rows * m.nV[lp] * sizeof(double) +
                             nmp * m.gcols[lp] * sizeof(double) + (kRpow + kMaxPb) * sizeof(double) +
                             (size_t)m.gcols[lp] * sizeof(int2);
        if ((int)bytes > best) best = (int)bytes;
    }
    return best;
}

bool stage_rows_fit(const Meta& m, int rows) { return phase3_fits(rows, 2 * m.l_max + 1); }

int chunk_smem_bytes(const Meta& m, int rows) {
    int best = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        const size_t nmp = 2 * lp + 1;
        const size_t bytes = m.n_xs * sizeof(double2) + (size_t)rows * m.gcols[lp] * sizeof(double2) +
                             (size_t)m.n_f * sizeof(double2) + (size_t)rows * m.nV[lp] * sizeof(double) +
                             nmp * m.gcols[lp] * sizeof(double) + (kRpow + kMaxPb) * sizeof(double) +
                             (size_t)m.gcols[lp] * sizeof(int2) + (size_t)m.nV[lp] * sizeof(int);
        if ((int)bytes > best) best = (int)bytes;
    }
    return best;
}

// The dynamic-LDS attribute is per kernel and process-wide: it is only ever
// raised (to the largest size any plan has asked for), so that a plan created
// later with a smaller basis does not lower it under an earlier plan's launches.
hipError_t stage_set_smem_limit(int, int bytes) {
    static std::mutex mu;
    static int set_bytes = 0;
    std::lock_guard<std::mutex> lk(mu);
    if (bytes <= set_bytes) return hipSuccess;
#define WPCCC_FN_PAIR(R)                                                                        \
    (const void*)k_stage<R, false, false>, (const void*)k_stage<R, false, true>,                 \
        (const void*)k_stage<R, true, true>, (const void*)k_stage<R, true, false>, (const void*)k_chunk<R>,
#define WPCCC_FN_GG(R) (const void*)k_stage<R, false, true, true>, (const void*)k_stage<R, true, true, true>,
    const void* fns[] = {WPCCC_STAGE_ROWS(WPCCC_FN_PAIR) WPCCC_STAGE_ROWS_GG(WPCCC_FN_GG)(const void*)k_apply<kRowsPerBlock>,
                         (const void*)k_apply<kApplyRowsLarge>, (const void*)k_apply<4, true>,
                         (const void*)k_apply<2, true>, (const void*)k_apply<1, true>};
#undef WPCCC_FN_PAIR
#undef WPCCC_FN_GG
    hipError_t e = hipSuccess;
    for (const void* f : fns)
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess) set_bytes = bytes;
    return e;
}

int chunk_grid(const Meta& hm, int n_traj, int rows) { return 8 * ((n_traj * stage_chunks(hm, rows) + 7) / 8); }

int stage_wgs_per_cu(int rows, int smem) {
    const void* f = nullptr;
    switch (rows) {
#define WPCCC_CASE(R) \
    case R: f = (const void*)k_stage<R, false, false>; break;
        WPCCC_STAGE_ROWS(WPCCC_CASE)
#undef WPCCC_CASE
        default: return 0;
    }
    int dev = 0, per_cu = 0, lds_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kStageThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    // the occupancy query without dynamic LDS (above 64 KiB it would need the
    // kernel attribute first), then the LDS bound
    return smem > 0 ? std::min(per_cu, lds_cu / smem) : per_cu;
}

static const void* chunk_fn(int rows) {
    switch (rows) {
#define WPCCC_CASE(R) \
    case R: return (const void*)k_chunk<R>;
        WPCCC_STAGE_ROWS(WPCCC_CASE)
#undef WPCCC_CASE
        default: return nullptr;
    }
}

bool chunk_fits(const Meta& hm, int n_traj, int rows, int smem) {
    int dev = 0, n_cu = 0, per_cu = 0, coop = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
    if (!chunk_fn(rows)) return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, chunk_fn(rows), kStageThreads, smem) != hipSuccess)
        return false;
    return (long long)per_cu * n_cu >= chunk_grid(hm, n_traj, rows);
}

hipError_t launch_chunk(const ChunkArgs& a, const Meta& hm, int smem, int rows, hipStream_t st, const LaunchEv& ev) {
    const dim3 grid(chunk_grid(hm, a.n_traj, rows)), block(kStageThreads);
    ChunkArgs arg = a;
    void* params[] = {&arg};
    if (ev.a) (void)hipEventRecord(ev.a, st);
    if (!chunk_fn(rows)) return hipErrorInvalidValue;
    const hipError_t e = hipLaunchCooperativeKernel(chunk_fn(rows), grid, block, params, smem, st);
    if (ev.b) (void)hipEventRecord(ev.b, st);
    return e;
}

hipError_t launch_apply(const ApplyArgs& a, int n_ops, const Meta& hm, int n_traj_launch, int smem, int rows,
                        bool gg, hipStream_t st, const LaunchEv& ev) {
    const dim3 grid(stage_chunks(hm, rows), n_traj_launch, n_ops);
    if (gg) {
        if (rows == 4) WPCCC_LAUNCH(ev, (k_apply<4, true>), grid, dim3(kStageThreads), smem, st, a);
        else if (rows == 2) WPCCC_LAUNCH(ev, (k_apply<2, true>), grid, dim3(kStageThreads), smem, st, a);
        else if (rows == 1) WPCCC_LAUNCH(ev, (k_apply<1, true>), grid, dim3(kStageThreads), smem, st, a);
        else return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (rows == kRowsPerBlock)
        WPCCC_LAUNCH(ev, k_apply<kRowsPerBlock>, grid, dim3(kStageThreads), smem, st, a);
    else if (rows == kApplyRowsLarge)
        WPCCC_LAUNCH(ev, k_apply<kApplyRowsLarge>, grid, dim3(kStageThreads), smem, st, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_chunk_counter(int* chunk, int reset, hipStream_t st) {
    hipLaunchKernelGGL(k_chunk_counter, dim3(1), dim3(1), 0, st, chunk, reset);
    return hipGetLastError();
}

hipError_t launch_grad_sum(const double* gpart, int n_part, double* grad, int n_traj, hipStream_t st) {
    hipLaunchKernelGGL(k_grad_sum, dim3(n_traj), dim3(64), 0, st, gpart, n_part, grad);
    return hipGetLastError();
}

hipError_t launch_table_nodes(const double2* tab, const int* dl, int n_frow, int n_r, double r_max, double* out,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_table_nodes, dim3((n_frow + 255) / 256, n_r + 1), dim3(256), 0, st, tab, dl, n_frow, n_r,
                       r_max, out);
    return hipGetLastError();
}

hipError_t launch_table_f32(const double2* tab, const int* dl, int n_frow, int n_r, double r_max, float2* out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_table_f32, dim3((n_frow + 255) / 256, n_r + 1), dim3(256), 0, st, tab, dl, n_frow, n_r, r_max,
                       out);
    return hipGetLastError();
}

hipError_t launch_table_shift(double2* tab, int n_frow, int n_r, const int* idx, const double* val, int count,
                              hipStream_t st) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_table_shift, dim3((count + 255) / 256, n_r + 1), dim3(256), 0, st, tab, n_frow, idx, val,
                       count);
    return hipGetLastError();
}

hipError_t launch_moments(const double* r, const double* w, const double* phiT, const int* da, const int* db,
                          const int* dl, int n_r, int n_f, int n_frow, double2* tab, hipStream_t st) {
    const int nb = (n_frow + 127) / 128;
    hipLaunchKernelGGL(k_moments, dim3(nb), dim3(128), 0, st, r, w, phiT, da, db, dl, n_r, n_f, n_frow, tab);
    return hipGetLastError();
}

hipError_t launch_prologue(const PrologueArgs& a, int n_traj_launch, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_prologue, dim3(a.n, n_traj_launch), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_slot_setup(const SetupArgs& a, const Meta& hm, hipStream_t st, const LaunchEv& ev) {
    const int nbG = (hm.n_g + 255) / 256;
    WPCCC_LAUNCH(ev, k_slot_setup, dim3(a.nbF + a.nbP + nbG), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& a, const Meta& hm, int n_traj_launch, int smem, hipStream_t st, const LaunchEv& ev,
                        int rows) {
    const dim3 grid(8 * ((n_traj_launch * a.nwg + 7) / 8)), block(kStageThreads);
    StageArgs a1 = a;
    a1.n_paths = n_traj_launch;
    if (a.gg) {
        // large bases: cached F, angular factors from global memory
        if (!a.fc_cur) return hipErrorInvalidValue;
        switch (rows) {
#define WPCCC_CASE(R)                                                                                        \
    case R:                                                                                                  \
        if (a.tb.tab32) WPCCC_LAUNCH(ev, (k_stage<R, true, true, true>), grid, block, smem, st, a1);       \
        else WPCCC_LAUNCH(ev, (k_stage<R, false, true, true>), grid, block, smem, st, a1);                  \
        break;
            WPCCC_STAGE_ROWS_GG(WPCCC_CASE)
#undef WPCCC_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (rows) {
#define WPCCC_CASE(R)                                                                    \
    case R:                                                                              \
        if (a.tb.tab32 && a.fc_cur) WPCCC_LAUNCH(ev, (k_stage<R, true, true>), grid, block, smem, st, a1); \
        else if (a.tb.tab32) WPCCC_LAUNCH(ev, (k_stage<R, true, false>), grid, block, smem, st, a1);       \
        else if (a.fc_cur) WPCCC_LAUNCH(ev, (k_stage<R, false, true>), grid, block, smem, st, a1);       \
        else WPCCC_LAUNCH(ev, (k_stage<R, false, false>), grid, block, smem, st, a1);                    \
        break;
        WPCCC_STAGE_ROWS(WPCCC_CASE)
#undef WPCCC_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fpoint(const Meta* m, const Meta& hm, const Tables& tb, const PointArrays& pt, int p, int traj0,
                         int n_paths, void* fc, hipStream_t st, const LaunchEv& ev) {
    const dim3 grid((hm.n_frow + 255) / 256, n_paths);
    if (tb.tab32) WPCCC_LAUNCH(ev, k_fpoint<true>, grid, dim3(256), 0, st, m, tb, pt, p, traj0, fc);
    else WPCCC_LAUNCH(ev, k_fpoint<false>, grid, dim3(256), 0, st, m, tb, pt, p, traj0, fc);
    return hipGetLastError();
}

hipError_t launch_couplings_dense(const Meta* m, const Meta& hm, const double* Frow, const double* G,
                                  const double2* PH, double Zp, double2* H, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_couplings_dense, dim3((hm.n_states + 127) / 128, hm.n_states), dim3(128), 0, st, m, Frow,
                       G, PH, Zp, H);
    return hipGetLastError();
}

hipError_t launch_probabilities(const double2* X, int n_traj, int n_states, int n_pad, double* P, double* norm,
                                hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_probabilities, dim3(n_traj), dim3(256), 0, st, X, n_states, n_pad, P, norm);
    return hipGetLastError();
}

}  // namespace wpccc

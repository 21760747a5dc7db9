// HIP kernels of the two-centre path on gfx950.
//
// Per new coupling position (z_mid, z_new of Algorithm 1) and path:
//   k_2c_nodes     spheroidal nodes (eta, tau) of Eq. K2 at this R: r_A, r_B,
//                  angles, the phase (v z / 2) eta tau, Bessel J_m(X), the
//                  quadrature weight times each potential weight, and the
//                  five-point interpolation stencils at r_A and r_B
//   k_2c_contract  the Eq. K2 integrals as dense real contractions on MFMA
//                  (v_mfma_f64_16x16x4): for molecular |q'| = s, |q| = t,
//                  T[k][a][b] = sum_p A_s[a](p) B_t[b](p) w_k(p) with
//                  A_s[a](p) = f_a(r_A) Pbar_{l_a}^s(cos theta_A), B likewise,
//                  w_k = omega W J_m(X) {cos, sin}((v z / 2) eta tau)
//   k_2c_assemble  Eq. K1: signs of negative q', q and J_{-m}, (-i)^(q-q'),
//                  the Eq. K2 prefactor and the Wigner rotation to the lab
//                  frame, interaction phases -> K, Q blocks of S and H
//   k_setup_batch, k_2c_direct   D_T and D_P blocks (Eq. D1 on each centre)
//   k_lu           LU with partial pivoting of S (LAPACK conventions)
// Per RK4 stage: k_2c_stage  y = S^{-1} (H u), K = -(i/v) y and the RK4 update.
#include <hip/hip_runtime.h>

#include "plan2c.h"

namespace wpccc {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline void job_of(const Jobs& J, int y, int& pl, int& slot, double& z) {
    pl = J.path0 + y / J.n_sub;
    const int sub = y % J.n_sub;
    slot = J.slot[sub];
    z = J.z[sub];
}

// Lagrange weights at r for the nodes j0..j0+4 of r_i = rmax (i/nr)^2, j0 + 2
// the node nearest in sqrt(r/rmax); returns j0, or -1 when r > rmax.
__device__ inline int lagrange5(double r, double rmax, int nr, double* L) {
    if (!(r <= rmax)) {
        for (int i = 0; i < 5; ++i) L[i] = 0.0;
        return -1;
    }
    int j = (int)rint(nr * sqrt(r / rmax));
    j = max(2, min(nr - 2, j));
    double rn[5];
    for (int i = 0; i < 5; ++i) {
        const double x = (double)(j - 2 + i) / nr;
        rn[i] = rmax * x * x;
    }
    for (int i = 0; i < 5; ++i) {
        double p = 1.0;
        for (int q = 0; q < 5; ++q)
            if (q != i) p *= (r - rn[q]) / (rn[i] - rn[q]);
        L[i] = p;
    }
    return j - 2;
}

// Pbar_l^m(x) = sqrt((l-m)!/(l+m)!) P_l^m(x), Condon-Shortley phase, 0 <= m <= l.
__device__ inline double pbar(int l, int m, double x) {
    const double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int i = 1; i <= m; ++i) pmm *= -sqrt((2.0 * i - 1.0) / (2.0 * i)) * s;
    if (l == m) return pmm;
    double p0 = pmm, p1 = sqrt(2.0 * m + 1.0) * x * pmm;
    for (int ll = m + 1; ll < l; ++ll) {
        const double p2 = ((2.0 * ll + 1.0) * x * p1 - sqrt((double)(ll + m) * (ll - m)) * p0) /
                          sqrt((double)(ll + 1 + m) * (ll + 1 - m));
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

__global__ __launch_bounds__(256) void k_2c_nodes(NodeArgs a) {
    const Meta2C& m = *a.m;
    int pl, slot;
    double z;
    job_of(a.jobs, blockIdx.y, pl, slot, z);
    const int j = a.paths[pl];
    const double b = a.bvec[j], v = a.vvec[j];
    const double R = sqrt(b * b + z * z);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // beyond x = rmaxT + rmaxP - R one of r_A, r_B exceeds its grid: f = 0
        const double lim = (m.rmaxT + m.rmaxP - R) * (1.0 + 1e-12) + 1e-12;
        int na = 0;
        while (na < m.n_eta && a.xlag[na] <= lim) ++na;
        a.n_act[blockIdx.y] = na * m.n_tau;
    }
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m.n_nodes) return;
    const int ie = p / m.n_tau, it = p - ie * m.n_tau;
    const double eta = 1.0 + a.xlag[ie] / R, tau = a.tleg[it];
    const double om = a.wlag[ie] / R * a.wleg[it];
    const double rA = R * (eta + tau) / 2.0, rB = R * (eta - tau) / 2.0;
    const double cA = (1.0 + eta * tau) / (eta + tau), cB = (eta * tau - 1.0) / (eta - tau);
    const double X = (v * b / 2.0) * sqrt(fmax(0.0, (eta * eta - 1.0) * (1.0 - tau * tau)));
    double sn, cs;
    sincos((v * z / 2.0) * eta * tau, &sn, &cs);
    const size_t nn = m.n_nodes;
    double* nd = a.nodes + (size_t)blockIdx.y * m.n_fields * nn;
    int* js = a.jst + (size_t)blockIdx.y * 2 * nn;
    nd[0 * nn + p] = rA;
    nd[1 * nn + p] = rB;
    nd[2 * nn + p] = cA;
    nd[3 * nn + p] = cB;
    nd[4 * nn + p] = cs;
    nd[5 * nn + p] = sn;
    nd[6 * nn + p] = om * (eta * eta - tau * tau);
    nd[7 * nn + p] = om * (-(2.0 * m.ZT / R) * (eta - tau));
    nd[8 * nn + p] = om * (-(2.0 * m.ZP / R) * (eta + tau));
    double L[5];
    js[p] = lagrange5(rA, m.rmaxT, m.nrT, L);
    for (int i = 0; i < 5; ++i) nd[(9 + i) * nn + p] = L[i];
    js[nn + p] = lagrange5(rB, m.rmaxP, m.nrP, L);
    for (int i = 0; i < 5; ++i) nd[(14 + i) * nn + p] = L[i];
    for (int q = 0; q <= 2 * m.L; ++q) nd[(kNodeFixed + q) * nn + p] = jn(q, X);
}

constexpr int kMaxFields = kNodeFixed + 2 * kMaxL + 1;

// grid: x = tile (s, t, a0, b0), y = job.  Four waves; each wave owns nk/2
// column tiles of 16 (B' columns k*32 + b) for both 16-row halves of the tile.
__global__ __launch_bounds__(256) void k_2c_contract(ContractArgs a) {
    extern __shared__ double Bs[];  // [kNodeChunk][32 * nk]
    __shared__ double As[kNodeChunk][kTile];
    __shared__ double nf[kNodeChunk][kMaxFields];
    __shared__ int jA[kNodeChunk], jB[kNodeChunk];
    __shared__ double PbA[kNodeChunk][kMaxL + 1], PbB[kNodeChunk][kMaxL + 1];
    __shared__ double wk[kNodeChunk][kMaxK];
    const Meta2C& m = *a.m;
    const int y = blockIdx.y;
    const int2 tl = a.tiles[blockIdx.x];
    const int s = tl.x & 0xff, t = tl.x >> 8, a0 = tl.y & 0xffff, b0 = tl.y >> 16;
    const int n_w = m.n_w;
    const int nk = st_nk(s, t, n_w);
    const int o1 = abs(s - t), o2 = s + t;
    const int nA = m.nA[s], nB = m.nB[t];
    const int nF = m.n_fields;
    const size_t nn = m.n_nodes;
    const double* nd = a.nodes + (size_t)y * nF * nn;
    const int* js = a.jst + (size_t)y * 2 * nn;
    const int nact = a.n_act[y];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int n_nt = nk / 2;
    const int nrow = kTile * nk;

    dbl4 acc[kMaxK];
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};

    for (int base = 0; base < nact; base += kNodeChunk) {
        for (int e = tid; e < kNodeChunk * nF; e += blockDim.x) {
            const int k = e % kNodeChunk, f = e / kNodeChunk;
            const int p = base + k;
            nf[k][f] = (p < nact) ? nd[(size_t)f * nn + p] : 0.0;
        }
        if (tid < 2 * kNodeChunk) {
            const int k = tid % kNodeChunk, side = tid / kNodeChunk;
            const int p = base + k;
            const int jv = (p < nact) ? js[side * nn + p] : -1;
            if (side == 0) jA[k] = jv;
            else jB[k] = jv;
        }
        __syncthreads();
        for (int e = tid; e < kNodeChunk * (kMaxL + 1) * 2; e += blockDim.x) {
            const int side = e / (kNodeChunk * (kMaxL + 1));
            const int rem = e - side * kNodeChunk * (kMaxL + 1);
            const int k = rem / (kMaxL + 1), l = rem - k * (kMaxL + 1);
            if (side == 0) {
                if (l >= s && l <= m.LT) PbA[k][l] = pbar(l, s, nf[k][2]);
            } else {
                if (l >= t && l <= m.LP) PbB[k][l] = pbar(l, t, nf[k][3]);
            }
        }
        for (int e = tid; e < kNodeChunk * nk; e += blockDim.x) {
            const int k = e / nk, kk = e - k * nk;
            const int order = kk / (2 * n_w), trig = (kk / n_w) & 1, w = kk % n_w;
            const double J = nf[k][kNodeFixed + (order == 0 ? o1 : o2)];
            wk[k][kk] = J * (trig ? nf[k][5] : nf[k][4]) * nf[k][6 + w];
        }
        __syncthreads();
        for (int e = tid; e < kNodeChunk * kTile; e += blockDim.x) {
            const int k = e / kTile, r = e - k * kTile;
            const int i = a0 + r;
            double val = 0.0;
            if (i < nA && jA[k] >= 0) {
                const int arad = m.radT_off[s] + i;
                const double* f = a.phiT_T + (size_t)jA[k] * m.nfT + arad;
                const double fv = nf[k][9] * f[0] + nf[k][10] * f[m.nfT] + nf[k][11] * f[2 * m.nfT] +
                                  nf[k][12] * f[3 * m.nfT] + nf[k][13] * f[4 * m.nfT];
                val = fv * PbA[k][a.radl_T[arad]];
            }
            As[k][r] = val;
        }
        for (int e = tid; e < kNodeChunk * kTile; e += blockDim.x) {
            const int k = e / kTile, c = e - k * kTile;
            const int jj = b0 + c;
            double val = 0.0;
            if (jj < nB && jB[k] >= 0) {
                const int brad = m.radP_off[t] + jj;
                const double* f = a.phiT_P + (size_t)jB[k] * m.nfP + brad;
                const double fv = nf[k][14] * f[0] + nf[k][15] * f[m.nfP] + nf[k][16] * f[2 * m.nfP] +
                                  nf[k][17] * f[3 * m.nfP] + nf[k][18] * f[4 * m.nfP];
                val = fv * PbB[k][a.radl_P[brad]];
            }
            double* row = Bs + k * nrow;
            for (int kk = 0; kk < nk; ++kk) row[kk * kTile + c] = val * wk[k][kk];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kNodeChunk / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4), li = lane & 15;
            const double af0 = As[kr][li], af1 = As[kr][16 + li];
#pragma unroll
            for (int q = 0; q < kMaxK / 2; ++q) {
                if (q < n_nt) {
                    const int nt = wave + 4 * q;
                    const double bf = Bs[kr * nrow + nt * 16 + li];
                    acc[2 * q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af0, bf, acc[2 * q], 0, 0, 0);
                    acc[2 * q + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(af1, bf, acc[2 * q + 1], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // D[row][col] of a 16x16 tile: lane l, register r -> row 4 r + l / 16, col l % 16
    // (A[i][k] in lane i + 16 k and B[k][j] in lane j + 16 k, as loaded above)
    double* out = a.tmol + (size_t)y * m.n_tmol + m.st_off[s][t];
#pragma unroll
    for (int q = 0; q < kMaxK / 2; ++q) {
        if (q < n_nt) {
            const int nt = wave + 4 * q;
            const int kk = nt / 2, half = nt % 2;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = a0 + mt * 16 + 4 * r + (lane >> 4);
                    const int jj = b0 + half * 16 + (lane & 15);
                    if (i < nA && jj < nB) out[((size_t)kk * nA + i) * nB + jj] = acc[2 * q + mt][r];
                }
        }
    }
}

// Wigner d^l_{mq}(theta) by Wigner's sum (convention d^1_{10} = -sin(theta)/sqrt 2).
__device__ double wigner_d(int l, int mm, int q, double c, double s) {
    double fac[2 * kMaxL + 2];
    fac[0] = 1.0;
    for (int i = 1; i < 2 * kMaxL + 2; ++i) fac[i] = fac[i - 1] * i;
    const double pre = sqrt(fac[l + mm] * fac[l - mm] * fac[l + q] * fac[l - q]);
    double tot = 0.0;
    for (int k = max(0, q - mm); k <= min(l + q, l - mm); ++k) {
        const double den = fac[l + q - k] * fac[k] * fac[mm - q + k] * fac[l - mm - k];
        const int ec = 2 * l + q - mm - 2 * k, es = mm - q + 2 * k;
        double term = 1.0;
        for (int i = 0; i < ec; ++i) term *= c;
        for (int i = 0; i < es; ++i) term *= s;
        tot += (((mm - q + k) & 1) ? -term : term) / den;
    }
    return pre * tot;
}

__host__ __device__ constexpr int d_off(int l) { return l * (4 * l * l - 1) / 3; }

// grid: x = element blocks (target x projectile pairs, then the identity
// blocks of S), y = job.
__global__ __launch_bounds__(256) void k_2c_assemble(AssembleArgs a) {
    __shared__ double dt[d_off(kMaxL + 1)];
    const Meta2C& m = *a.m;
    int pl, slot;
    double z;
    job_of(a.jobs, blockIdx.y, pl, slot, z);
    const int j = a.paths[pl];
    const double b = a.bvec[j], v = a.vvec[j];
    const double R = sqrt(b * b + z * z);
    const int N = m.N, NT = m.NT, NP = m.NP;
    const size_t ps = ((size_t)pl * kSlots2C + slot) * (size_t)N * N;
    double2* S = a.S + ps;
    double2* LU = a.LU + ps;
    double2* H = a.H + ps;
    const int n_off_blocks = (NT * NP + blockDim.x - 1) / blockDim.x;
    if ((int)blockIdx.x >= n_off_blocks) {
        // identity blocks of S
        const int e = (blockIdx.x - n_off_blocks) * blockDim.x + threadIdx.x;
        int r, c;
        if (e < NT * NT) {
            r = e / NT;
            c = e - r * NT;
        } else if (e < NT * NT + NP * NP) {
            const int f = e - NT * NT;
            r = NT + f / NP;
            c = NT + f % NP;
        } else {
            return;
        }
        const double2 val = make_double2(r == c ? 1.0 : 0.0, 0.0);
        S[r + (size_t)c * N] = val;
        LU[r + (size_t)c * N] = val;
        return;
    }
    const double ct = z / R;
    const double ch = sqrt(fmax(0.0, (1.0 + ct) / 2.0)), sh = sqrt(fmax(0.0, (1.0 - ct) / 2.0));
    for (int e = threadIdx.x; e < d_off(m.L + 1); e += blockDim.x) {
        int l = 0;
        while (d_off(l + 1) <= e) ++l;
        const int rem = e - d_off(l);
        const int im = rem / (2 * l + 1), iq = rem - im * (2 * l + 1);
        dt[e] = wigner_d(l, im - l, iq - l, ch, sh);
    }
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NT * NP) return;
    const int al = e / NP, be = e - al * NP;
    int la = 0, lb = 0;
    while (la < m.LT && al >= m.stT_off[la + 1]) ++la;
    while (lb < m.LP && be >= m.stP_off[lb + 1]) ++lb;
    const int ra = al - m.stT_off[la], rb = be - m.stP_off[lb];
    const int ma = ra / m.n_lT[la] - la, na = ra % m.n_lT[la];
    const int mb = rb / m.n_lP[lb] - lb, nb = rb % m.n_lP[lb];
    const int arad = m.radT_off[la] + na, brad = m.radP_off[lb] + nb;
    const double* tm = a.tmol + (size_t)blockIdx.y * m.n_tmol;
    const int n_w = m.n_w;
    double acc[kMaxW][2];
    for (int w = 0; w < kMaxW; ++w) acc[w][0] = acc[w][1] = 0.0;
    for (int qa = -la; qa <= la; ++qa) {
        const int s = abs(qa);
        const double dA = dt[d_off(la) + (ma + la) * (2 * la + 1) + (qa + la)];
        const int is = arad - m.radT_off[s];
        for (int qb = -lb; qb <= lb; ++qb) {
            const int t = abs(qb);
            const double dB = dt[d_off(lb) + (mb + lb) * (2 * lb + 1) + (qb + lb)];
            const int jt = brad - m.radP_off[t];
            const int n = qb - qa, mabs = abs(n);
            const int order = (mabs == abs(s - t)) ? 0 : 1;
            double c = dA * dB;
            if (qa < 0 && (s & 1)) c = -c;
            if (qb < 0 && (t & 1)) c = -c;
            if (n < 0 && (mabs & 1)) c = -c;
            // (-i)^n
            const int n4 = ((n % 4) + 4) % 4;
            const double pr = (n4 == 0) ? 1.0 : (n4 == 2 ? -1.0 : 0.0);
            const double pi = (n4 == 1) ? -1.0 : (n4 == 3 ? 1.0 : 0.0);
            const int nBt = m.nB[t];
            const size_t blk = (size_t)m.nA[s] * nBt;
            const double* base = tm + m.st_off[s][t] + (size_t)is * nBt + jt;
            for (int w = 0; w < n_w; ++w) {
                const double tc = base[(size_t)((order * 2 + 0) * n_w + w) * blk];
                const double ts = base[(size_t)((order * 2 + 1) * n_w + w) * blk];
                acc[w][0] += c * (pr * tc - pi * ts);
                acc[w][1] += c * (pr * ts + pi * tc);
            }
        }
    }
    const double pref = (R * R * R / 16.0) * sqrt((2.0 * la + 1.0) * (2.0 * lb + 1.0));
    double sn, cs;
    sincos((a.epsT[al] - a.epsP[be]) * z / v, &sn, &cs);
    double2 val[kMaxW];
    for (int w = 0; w < n_w; ++w) {
        const double xr = pref * acc[w][0], xi = pref * acc[w][1];
        val[w] = make_double2(xr * cs - xi * sn, xr * sn + xi * cs);
    }
    const int row = al, col = NT + be;
    S[row + (size_t)col * N] = val[0];                          // K
    S[col + (size_t)row * N] = make_double2(val[0].x, -val[0].y);  // K^dagger
    LU[row + (size_t)col * N] = val[0];
    LU[col + (size_t)row * N] = make_double2(val[0].x, -val[0].y);
    H[(size_t)row * N + col] = val[1];                          // Q
    const double2 low = (m.q_prior && n_w > 2) ? val[2] : val[1];
    H[(size_t)col * N + row] = make_double2(low.x, -low.y);     // Q^dagger or the prior form
}

// grid: x = [nbF Frow blocks | nbP phase blocks | G blocks], y = job.
__global__ __launch_bounds__(256) void k_setup_batch(SetupBatchArgs a) {
    const Meta& m = *a.meta;
    const Tables& T = a.tb;
    int pl, slot;
    double z;
    job_of(a.jobs, blockIdx.y, pl, slot, z);
    const int j = a.paths[pl];
    const double b = T.bvec[j], v = T.vvec[j];
    const double R = sqrt(b * b + z * z);
    const int bx = blockIdx.x;
    const size_t y = blockIdx.y;
    if (bx < a.nbF) {
        const int d = bx * blockDim.x + threadIdx.x;
        if (d >= m.n_frow) return;
        int lp = 0;
        while (lp < m.l_max && d >= m.frow_off[lp + 1]) ++lp;
        const int e = (d - m.frow_off[lp]) % m.nV[lp];
        const int lam = T.col_lam[m.col_off[lp] + e];
        int k = (int)floor(m.n_r * sqrt(fmin(R / m.r_max, 1.0)));
        k = max(0, min(k, m.n_r));
        auto rk = [&](int q) {
            const double x = (double)q / m.n_r;
            return m.r_max * x * x;
        };
        while (k < m.n_r && rk(k + 1) <= R) ++k;
        while (k > 0 && rk(k) > R) --k;
        double Rl = 1.0;
        for (int q = 0; q < lam; ++q) Rl *= R;
        const double2 ab = T.tab[(size_t)k * m.n_frow + d];
        a.Frow[y * m.n_frow + d] = ab.x / (Rl * R) + ab.y * Rl;
        return;
    }
    if (bx < a.nbF + a.nbP) {
        const int i = (bx - a.nbF) * blockDim.x + threadIdx.x;
        if (i < m.n_states) {
            double sn, cs;
            sincos(T.eps[i] * z / v, &sn, &cs);
            a.PH[y * m.n_states + i] = make_double2(cs, sn);
        }
        return;
    }
    const int i = (bx - a.nbF - a.nbP) * blockDim.x + threadIdx.x;
    if (i >= m.n_g) return;
    const int p = T.gpb[i];
    double g = 0.0;
    if (p >= 0) {
        int lam = 0;
        while ((lam + 1) * (lam + 2) / 2 <= p) ++lam;
        const int mu = p - lam * (lam + 1) / 2;
        g = T.gcoef[i] * pbar(lam, mu, z / R);
        if (a.parity < 0 && (lam & 1)) g = -g;
    }
    a.G[y * m.n_g + i] = g;
}

// D_T (charge Z_P) into H[0:NT, 0:NT] and D_P (charge Z_T) into H[NT:, NT:].
// grid: x = element blocks over NT^2 + NP^2, y = job.
__global__ __launch_bounds__(256) void k_2c_direct(DirectArgs a) {
    const Meta2C& m2 = *a.m;
    int pl, slot;
    double z;
    job_of(a.jobs, blockIdx.y, pl, slot, z);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int NT = m2.NT, NP = m2.NP, N = m2.N;
    const Meta* mp;
    const double *Frow, *G;
    const double2* PH;
    int row, col, off;
    double Zc;
    const size_t y = blockIdx.y;
    if (e < NT * NT) {
        mp = a.mT;
        row = e / NT;
        col = e - row * NT;
        off = 0;
        Frow = a.FrowT + y * a.n_frowT;
        G = a.GT + y * a.n_gT;
        PH = a.PHT + y * NT;
        Zc = m2.ZP;
    } else if (e < NT * NT + NP * NP) {
        const int f = e - NT * NT;
        mp = a.mP;
        row = f / NP;
        col = f - row * NP;
        off = NT;
        Frow = a.FrowP + y * a.n_frowP;
        G = a.GP + y * a.n_gP;
        PH = a.PHP + y * NP;
        Zc = m2.ZT;
    } else {
        return;
    }
    const Meta& m = *mp;
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
    const double wr = pr.x * pc.x + pr.y * pc.y, wi = pr.y * pc.x - pr.x * pc.y;  // pr conj(pc)
    const size_t ps = ((size_t)pl * kSlots2C + slot) * (size_t)N * N;
    a.H[ps + (size_t)(off + row) * N + off + col] = make_double2(Zc * acc * wr, Zc * acc * wi);
}

// LU with partial pivoting (ties: lowest row), column-major, one workgroup per matrix.
__global__ __launch_bounds__(256) void k_lu(LUArgs a) {
    __shared__ double rv[256];
    __shared__ int ri[256];
    int pl, slot;
    double z;
    job_of(a.jobs, blockIdx.x, pl, slot, z);
    const int N = a.N;
    double2* A = a.LU + ((size_t)pl * kSlots2C + slot) * (size_t)N * N;
    int* piv = a.piv + ((size_t)pl * kSlots2C + slot) * N;
    const int tid = threadIdx.x;
    for (int k = 0; k < N; ++k) {
        double best = -1.0;
        int bi = N;
        for (int i = k + tid; i < N; i += blockDim.x) {
            const double2 x = A[i + (size_t)k * N];
            const double mag = x.x * x.x + x.y * x.y;
            if (mag > best) {
                best = mag;
                bi = i;
            }
        }
        rv[tid] = best;
        ri[tid] = bi;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if (tid < o) {
                const double v2 = rv[tid + o];
                const int i2 = ri[tid + o];
                if (v2 > rv[tid] || (v2 == rv[tid] && i2 < ri[tid])) {
                    rv[tid] = v2;
                    ri[tid] = i2;
                }
            }
            __syncthreads();
        }
        const int p = ri[0];
        const double pmag = rv[0];
        __syncthreads();
        if (tid == 0) piv[k] = (pmag > 0.0) ? p : k;
        if (!(pmag > 0.0)) {
            if (tid == 0 && atomicCAS(&a.flag[1], 0, a.paths[pl] + 1) == 0) a.flag[2] = k;
            continue;
        }
        if (p != k)
            for (int c = tid; c < N; c += blockDim.x) {
                const double2 t0 = A[k + (size_t)c * N];
                A[k + (size_t)c * N] = A[p + (size_t)c * N];
                A[p + (size_t)c * N] = t0;
            }
        __syncthreads();
        const double2 d = A[k + (size_t)k * N];
        const double dn = d.x * d.x + d.y * d.y;
        const double2 inv = make_double2(d.x / dn, -d.y / dn);
        for (int i = k + 1 + tid; i < N; i += blockDim.x) {
            const double2 x = A[i + (size_t)k * N];
            A[i + (size_t)k * N] = make_double2(x.x * inv.x - x.y * inv.y, x.x * inv.y + x.y * inv.x);
        }
        __syncthreads();
        for (int c = k + 1; c < N; ++c) {
            const double2 u = A[k + (size_t)c * N];
            for (int i = k + 1 + tid; i < N; i += blockDim.x) {
                const double2 l = A[i + (size_t)k * N];
                double2 x = A[i + (size_t)c * N];
                x.x -= l.x * u.x - l.y * u.y;
                x.y -= l.x * u.y + l.y * u.x;
                A[i + (size_t)c * N] = x;
            }
        }
        __syncthreads();
    }
}

// One RK4 stage of one path: y = H u, y <- S^{-1} y (pivots, L, U), K = -(i/v) y.
__global__ __launch_bounds__(256) void k_2c_stage(Stage2CArgs a) {
    extern __shared__ double2 sm[];  // u [N], y [N]
    const int pl = blockIdx.x;
    const int j = a.paths[pl];
    const int N = a.N, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const size_t ps = ((size_t)pl * kSlots2C + a.slot) * (size_t)N * N;
    const double2* H = a.H + ps;
    const double2* LU = a.LU + ps;
    const int* piv = a.piv + ((size_t)pl * kSlots2C + a.slot) * N;
    double2* us = sm;
    double2* ys = sm + N;
    const double2* u = a.u_in + (size_t)j * a.n_pad;
    for (int i = tid; i < N; i += blockDim.x) us[i] = u[i];
    __syncthreads();
    for (int r = wave; r < N; r += blockDim.x >> 6) {
        const double2* hr = H + (size_t)r * N;
        double re = 0.0, im = 0.0;
        for (int c = lane; c < N; c += 64) {
            const double2 h = hr[c], x = us[c];
            re += h.x * x.x - h.y * x.y;
            im += h.x * x.y + h.y * x.x;
        }
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_xor(re, off, 64);
            im += __shfl_xor(im, off, 64);
        }
        if (lane == 0) ys[r] = make_double2(re, im);
    }
    __syncthreads();
    if (tid == 0)
        for (int k = 0; k < N; ++k) {
            const int p = piv[k];
            if (p != k) {
                const double2 t0 = ys[k];
                ys[k] = ys[p];
                ys[p] = t0;
            }
        }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
        const double2 yk = ys[k];
        for (int i = k + 1 + tid; i < N; i += blockDim.x) {
            const double2 l = LU[i + (size_t)k * N];
            ys[i].x -= l.x * yk.x - l.y * yk.y;
            ys[i].y -= l.x * yk.y + l.y * yk.x;
        }
        __syncthreads();
    }
    for (int k = N - 1; k >= 0; --k) {
        if (tid == 0) {
            const double2 d = LU[k + (size_t)k * N], x = ys[k];
            const double dn = d.x * d.x + d.y * d.y;
            ys[k] = make_double2((x.x * d.x + x.y * d.y) / dn, (x.y * d.x - x.x * d.y) / dn);
        }
        __syncthreads();
        const double2 yk = ys[k];
        for (int i = tid; i < k; i += blockDim.x) {
            const double2 uu = LU[i + (size_t)k * N];
            ys[i].x -= uu.x * yk.x - uu.y * yk.y;
            ys[i].y -= uu.x * yk.y + uu.y * yk.x;
        }
        __syncthreads();
    }
    const double sc = 1.0 / a.vvec[j];
    const double h = a.h;
    for (int i = tid; i < N; i += blockDim.x) {
        const double2 yy = ys[i];
        const double2 K = make_double2(sc * yy.y, -sc * yy.x);  // -(i/v) y
        const size_t oi = (size_t)j * a.n_pad + i;
        const double2 x0 = a.X[oi];
        if (a.stage == 1) {
            a.u_out[oi] = make_double2(x0.x + 0.5 * h * K.x, x0.y + 0.5 * h * K.y);
            a.Xacc[oi] = make_double2(x0.x + h / 6.0 * K.x, x0.y + h / 6.0 * K.y);
        } else if (a.stage == 2 || a.stage == 3) {
            const double c = (a.stage == 2) ? 0.5 * h : h;
            a.u_out[oi] = make_double2(x0.x + c * K.x, x0.y + c * K.y);
            const double2 xa = a.Xacc[oi];
            a.Xacc[oi] = make_double2(xa.x + h / 3.0 * K.x, xa.y + h / 3.0 * K.y);
        } else {
            const double2 xa = a.Xacc[oi];
            const double2 xn = make_double2(xa.x + h / 6.0 * K.x, xa.y + h / 6.0 * K.y);
            if (!isfinite(xn.x) || !isfinite(xn.y)) atomicOr(a.flag, 1);
            a.X[oi] = xn;
        }
    }
}

// P = |X|^2 and X^dagger S X (S column-major) per path.
__global__ __launch_bounds__(256) void k_2c_finish(const double2* __restrict__ X, const double2* __restrict__ S,
                                                   int N, int n_pad, const int* __restrict__ paths, int slot,
                                                   double* __restrict__ P, double* __restrict__ norm) {
    __shared__ double red[256];
    const int pl = blockIdx.x;
    const int j = paths[pl];
    const double2* x = X + (size_t)j * n_pad;
    const double2* Sm = S + ((size_t)pl * kSlots2C + slot) * (size_t)N * N;
    double acc = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double yr = 0.0, yi = 0.0;
        for (int c = 0; c < N; ++c) {
            const double2 s = Sm[i + (size_t)c * N], xc = x[c];
            yr += s.x * xc.x - s.y * xc.y;
            yi += s.x * xc.y + s.y * xc.x;
        }
        const double2 xi = x[i];
        acc += xi.x * yr + xi.y * yi;
        if (P) P[(size_t)j * n_pad + i] = xi.x * xi.x + xi.y * xi.y;
    }
    if (P)
        for (int i = N + threadIdx.x; i < n_pad; i += blockDim.x) P[(size_t)j * n_pad + i] = 0.0;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && norm) norm[j] = red[0];
}

__global__ void k_transpose_copy(const double2* __restrict__ src, double2* __restrict__ dst, int N) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c < N) dst[(size_t)r * N + c] = src[r + (size_t)c * N];
}

}  // namespace

int contract_smem_bytes(int n_w) { return kNodeChunk * kTile * 4 * n_w * (int)sizeof(double); }

hipError_t contract_set_smem(int bytes) {
    return hipFuncSetAttribute((const void*)k_2c_contract, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

hipError_t launch_2c_nodes(const NodeArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st) {
    hipLaunchKernelGGL(k_2c_nodes, dim3((hm.n_nodes + 255) / 256, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_contract(const ContractArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st) {
    hipLaunchKernelGGL(k_2c_contract, dim3(hm.n_tiles, n_jobs), dim3(256), contract_smem_bytes(hm.n_w), st, a);
    return hipGetLastError();
}

hipError_t launch_2c_assemble(const AssembleArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st) {
    const int nb = (hm.NT * hm.NP + 255) / 256 + (hm.NT * hm.NT + hm.NP * hm.NP + 255) / 256;
    hipLaunchKernelGGL(k_2c_assemble, dim3(nb, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_setup_batch(const SetupBatchArgs& a, const Meta& hm, int n_jobs, hipStream_t st) {
    const int nbG = (hm.n_g + 255) / 256;
    hipLaunchKernelGGL(k_setup_batch, dim3(a.nbF + a.nbP + nbG, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_direct(const DirectArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st) {
    const int nb = (hm.NT * hm.NT + hm.NP * hm.NP + 255) / 256;
    hipLaunchKernelGGL(k_2c_direct, dim3(nb, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lu(const LUArgs& a, int n_jobs, hipStream_t st) {
    hipLaunchKernelGGL(k_lu, dim3(n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_stage(const Stage2CArgs& a, int n_paths, hipStream_t st) {
    hipLaunchKernelGGL(k_2c_stage, dim3(n_paths), dim3(256), 2 * a.N * sizeof(double2), st, a);
    return hipGetLastError();
}

hipError_t launch_2c_finish(const double2* X, const double2* S, int N, int n_pad, const int* paths, int n_paths,
                            int slot, double* P, double* norm, hipStream_t st) {
    hipLaunchKernelGGL(k_2c_finish, dim3(n_paths), dim3(256), 0, st, X, S, N, n_pad, paths, slot, P, norm);
    return hipGetLastError();
}

hipError_t launch_transpose_copy(const double2* src, double2* dst, int N, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_copy, dim3((N + 255) / 256, N), dim3(256), 0, st, src, dst, N);
    return hipGetLastError();
}

}  // namespace wpccc

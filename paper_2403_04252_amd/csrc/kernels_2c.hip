// HIP kernels of the two-centre path on gfx950.
//
// Per new coupling position (z_mid, z_new of Algorithm 1) and path:
//   k_2c_nodes     spheroidal nodes (eta, tau) of Eq. K2 at this R: the phase
//                  (v z / 2) eta tau, Bessel J_m(X), the quadrature weight
//                  times each potential weight, the five-point interpolation
//                  stencils at r_A and r_B and Pbar_l^m at theta_A, theta_B
//   k_2c_contract  the Eq. K2 integrals as dense real contractions on MFMA
//                  (v_mfma_f64_16x16x4): for molecular |q'| = s, |q| = t,
//                  T[k][a][b] = sum_p A_s[a](p) B_t[b](p) w_k(p) with
//                  A_s[a](p) = f_a(r_A) Pbar_{l_a}^s(cos theta_A), B likewise,
//                  w_k = omega W J_m(X) {cos, sin}((v z / 2) eta tau)
//   k_2c_assemble  Eq. K1: signs of negative q', q and J_{-m}, (-i)^(q-q'),
//                  the Eq. K2 prefactor and the Wigner rotation to the lab
//                  frame, interaction phases -> K, Q blocks of S and H
//   k_setup_batch, k_2c_direct   D_T and D_P blocks (Eq. D1 on each centre)
// Per RK4 stage: k_2c_hu  y = P (H u) over many workgroups per path, then
// k_2c_solve  y <- U^{-1} L^{-1} y, K = -(i/v) y and the RK4 update (in the
// explicit form y = M u with M = S^{-1} H formed per coupling point, and
// k_2c_solve only updates).
// The LU factorisation of S is in kernels_lu.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "plan2c.h"

namespace wpccc {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline void job_of(const Jobs& J, int y, int& pl, int& slot, double& z) {
    pl = J.path0 + y / J.n_sub;
    const int sub = y % J.n_sub;
    slot = J.slot[sub];
    z = J.zdev ? J.zdev[3 * (size_t)(*J.step + J.ahead) + sub] : J.z[sub];
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
    nd[kFCos * nn + p] = cs;
    nd[kFSin * nn + p] = sn;
    nd[(kFW + 0) * nn + p] = om * (eta * eta - tau * tau);
    nd[(kFW + 1) * nn + p] = om * (-(2.0 * m.ZT / R) * (eta - tau));
    nd[(kFW + 2) * nn + p] = om * (-(2.0 * m.ZP / R) * (eta + tau));
    double L[5];
    js[p] = lagrange5(rA, m.rmaxT, m.nrT, L);
    for (int i = 0; i < 5; ++i) nd[(kFLA + i) * nn + p] = L[i];
    js[nn + p] = lagrange5(rB, m.rmaxP, m.nrP, L);
    for (int i = 0; i < 5; ++i) nd[(kFLB + i) * nn + p] = L[i];
    for (int q = 0; q <= 2 * m.L; ++q) nd[(kFJ + q) * nn + p] = jn(q, X);
    for (int l = 0; l <= m.LT; ++l)
        for (int mm = 0; mm <= l; ++mm) nd[(m.f_pa + l * (l + 1) / 2 + mm) * nn + p] = pbar(l, mm, cA);
    for (int l = 0; l <= m.LP; ++l)
        for (int mm = 0; mm <= l; ++mm) nd[(m.f_pb + l * (l + 1) / 2 + mm) * nn + p] = pbar(l, mm, cB);
}

// Interpolated operands of one position.  grid: x = blocks of 64 nodes,
// y = blocks of 64 radial functions (side T, then side P), z = job.  Each wave
// takes 16 nodes; per node its 64 lanes are 64 radial functions, so the five
// stencil values of consecutive functions are consecutive doubles of phiT
// (coalesced).  The interpolated f_a(r) of the 64 x 64 tile is formed once in
// LDS and written, times the Legendre factor, to the rows of every block s
// whose radial functions (l_a >= s) it holds, row by row with lanes over
// nodes.  The factors Pbar_l^s of the tile's l range (one contiguous range
// of node fields) are loaded into registers with the stencils, held while
// f_a(r) is formed and then staged in LDS over the stencil weights (dynamic
// LDS of interp_lds_bytes).
constexpr int kInterpPReg = 4;   // Legendre factors per thread held in registers
constexpr int kInterpMaxDynLds = 64 * 1024;   // at most 66 fields of 64 doubles (l <= 10)
template <typename T>
__global__ __launch_bounds__(256) void k_2c_interp(InterpArgs a) {
    __shared__ double tile[64][65];
    __shared__ int sj[64], sl[64];
    // stencil weights [64][5] until f_a(r) is formed, then the Legendre
    // factors [n_pf][64] (fields pb0 .. pb0 + n_pf - 1 of the side)
    extern __shared__ double dyn[];
    double (*sL)[5] = reinterpret_cast<double (*)[5]>(dyn);
    double* sP = dyn;
    const Meta2C& m = *a.m;
    const int y = blockIdx.z;
    const int nact = a.n_act[y];
    const int p0 = blockIdx.x * 64;
    if (p0 >= nact) return;
    const int nbT = (m.nfT + 63) / 64;
    const bool sideP = (int)blockIdx.y >= nbT;
    const int f0 = (sideP ? blockIdx.y - nbT : blockIdx.y) * 64;
    const int nf = sideP ? m.nfP : m.nfT;
    const int ls = sideP ? m.LP : m.LT;
    const int rows = sideP ? m.rowsP : m.rowsT;
    const int fP = sideP ? m.f_pb : m.f_pa;
    const int* rad_off = sideP ? m.radP_off : m.radT_off;
    const int* row_off = sideP ? m.rowP_off : m.rowT_off;
    const double* phiT = sideP ? a.phiT_P : a.phiT_T;
    const size_t nn = m.n_nodes;
    const double* nd = a.nodes + (size_t)y * m.n_fields * nn;
    const int* js = a.jst + (size_t)y * 2 * nn + (sideP ? nn : 0);
    const int fL = sideP ? kFLB : kFLA;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int fend = min(f0 + 64, nf);
    // l of the tile's first and last function (functions are ordered by l)
    int l_lo = 0, l_hi = 0;
    while (l_lo < ls && rad_off[l_lo + 1] <= f0) ++l_lo;
    while (l_hi < ls && rad_off[l_hi + 1] <= fend - 1) ++l_hi;
    // Legendre fields l (l + 1) / 2 + s for l_lo <= l <= l_hi, s <= l
    const int pb0 = l_lo * (l_lo + 1) / 2, n_pf = (l_hi + 1) * (l_hi + 2) / 2 - pb0;
    double pv[kInterpPReg];
#pragma unroll
    for (int r = 0; r < kInterpPReg; ++r) {
        const int e = tid + r * 256, k = e & 63, p = p0 + k;
        pv[r] = (e < n_pf * 64 && p < nact) ? nd[(size_t)(fP + pb0 + (e >> 6)) * nn + p] : 0.0;
    }
    // stencils of the 64 nodes, l of the 64 functions
    for (int e = tid; e < 64 * 5; e += blockDim.x) {
        const int k = e % 64, q = e / 64, p = p0 + k;
        sL[k][q] = (p < nact) ? nd[(size_t)(fL + q) * nn + p] : 0.0;
    }
    if (tid < 64) sj[tid] = (p0 + tid < nact) ? js[p0 + tid] : -1;
    if (tid >= 64 && tid < 128) {
        const int fa = f0 + tid - 64;
        int l = l_lo;
        while (l < l_hi && rad_off[l + 1] <= fa) ++l;
        sl[tid - 64] = l;
    }
    __syncthreads();
    // f_a(r) of function f0 + lane at the wave's 16 nodes
    const int fa = f0 + lane;
    for (int kk = 0; kk < 16; ++kk) {
        const int k = wave * 16 + kk;
        const int j = sj[k];
        double v = 0.0;
        if (fa < nf && j >= 0) {
            const double* f = phiT + (size_t)j * nf + fa;
            v = sL[k][0] * f[0] + sL[k][1] * f[nf] + sL[k][2] * f[2 * nf] + sL[k][3] * f[3 * nf] +
                sL[k][4] * f[4 * nf];
        }
        tile[lane][k] = v;
    }
    __syncthreads();
    // the Legendre factors over the stencil weights
#pragma unroll
    for (int r = 0; r < kInterpPReg; ++r)
        if (tid + r * 256 < n_pf * 64) sP[tid + r * 256] = pv[r];
    for (int e = tid + kInterpPReg * 256; e < n_pf * 64; e += blockDim.x) {
        const int k = e & 63, p = p0 + k;
        sP[e] = (p < nact) ? nd[(size_t)(fP + pb0 + (e >> 6)) * nn + p] : 0.0;
    }
    __syncthreads();
    // rows (s, a) for a in this tile and l_a >= s: functions [rad_off[s], nf)
    T* out = reinterpret_cast<T*>(sideP ? a.BT : a.AT) + (size_t)y * rows * nn;
    for (int s = 0; s <= l_hi; ++s) {
        const int alo = max(f0, rad_off[s]);
        const int cnt = fend - alo;
        const int rbase = row_off[s] + alo - rad_off[s];
        for (int e = tid; e < cnt * 64; e += blockDim.x) {
            const int k = e & 63, i = e >> 6, p = p0 + k, ti = alo - f0 + i, l = sl[ti];
            if (p < nact)
                out[(size_t)(rbase + i) * nn + p] =
                    sj[k] >= 0 ? (T)(tile[ti][k] * sP[(l * (l + 1) / 2 + s - pb0) * 64 + k]) : (T)0;
        }
    }
}

typedef float flt4 __attribute__((ext_vector_type(4)));

// Output row of register r in lane l of a 16 x 16 MFMA tile (column l % 16),
// measured on gfx950: 4 r + l / 16 for the FP64 instruction, 4 (l / 16) + r
// for the FP32 one.
__device__ inline int mfma_row_f64(int r, int l) { return 4 * r + (l >> 4); }
__device__ inline int mfma_row_f32(int r, int l) { return kF32RowByLaneGroup ? 4 * (l >> 4) + r : 4 * r + (l >> 4); }

constexpr int kWFields = 7;  // cos, sin, W_0..W_2, J_|s-t|, J_(s+t)
constexpr int kStageThreads2C = 256;  // threads of a contraction workgroup

// Work of one wave in a 32 x 32 tile with nk weights: KPW weights (kk0 ..
// kk0 + KPW - 1) times SPW of the four 16 x 16 subtiles.  SPW = 4: the wave
// covers the whole tile and kk0 = wave * KPW (nk = 4 KPW); SPW = 2: the wave
// covers the two subtiles of row half mt = wave / 2 and kk0 = (wave % 2) KPW
// (nk = 2 KPW).  One LDS read of an A value then serves 2 KPW products, one
// of a B value KPW * SPW / 2, and one of a weight SPW.
// LDS of a contraction workgroup.  As[node][row] and Bs[node][col] hold one
// chunk of operands at a row pitch of kPitch elements with the row index
// XOR-ed by 4 (node / 4): the MFMA reads (16 rows of 4 nodes per wave) and the
// staging writes (8 rows of 8 node quads per wave) then spread over the 64
// LDS banks with the fewest passes (pitch 40 for FP64, 48 for FP32).
template <typename T, int NC>
struct ContractLds {
    static constexpr int kPitch = sizeof(T) == 8 ? 40 : 48;
    T As[NC][kPitch], Bs[NC][kPitch];
    double fl[kWFields][NC];
    T wk[NC][kMaxK];   // weights w_k(p), formed in FP64 and stored in the product precision
};

// Nodes per chunk: kNodeChunk for FP64; twice that for the FP32 products,
// whose MFMA is three times faster, so that the per-chunk staging and the
// FP64 accumulation of the chunk sums are spread over more products.
template <bool MIXED>
constexpr int contract_chunk() { return MIXED ? 2 * kNodeChunk : kNodeChunk; }
__device__ inline int lds_swz(int node) { return 4 * ((node >> 2) & 7); }

// The MFMAs of one chunk for the wave's active subtiles: row halves
// mt0 .. mt0 + NA - 1 and column halves 0 .. NV - 1 (subtiles wholly outside
// the block are left out at compile time, so the k-step loop has no
// branches), KPW weights from kk0.  MIXED: FP32 products summed over the
// chunk in FP32 MFMA accumulators, then added to the FP64 ones.
template <bool MIXED, int KPW, int NMT, int NA, int NV, typename T, int NC>
__device__ __forceinline__ void chunk_mfma(const ContractLds<T, NC>& L, int mt0, int kk0, int li, int lk,
                                           bool r2, bool c2, dbl4 (&acc)[KPW][NMT][2]) {
    constexpr int NKS = NC / 4;
    T av[2][NA], bv[2][NV], w[2][KPW];
    auto load = [&](int ks, int b) {
        const int kr = ks * 4 + lk;
        const int sw = lds_swz(kr);
#pragma unroll
        for (int u = 0; u < NA; ++u) av[b][u] = L.As[kr][((mt0 + u) * 16 + li) ^ sw];
#pragma unroll
        for (int v = 0; v < NV; ++v) bv[b][v] = L.Bs[kr][(v * 16 + li) ^ sw];
#pragma unroll
        for (int i = 0; i < KPW; ++i) w[b][i] = L.wk[kr][kk0 + i];
    };
    if (!MIXED) {
        // FP64: one variant per weight split (NA = NMT, NV = 2) that skips
        // the second row half (!r2) and column half (!c2) at run time; an
        // FP64 MFMA is long enough that the branches cost little, and one
        // variant instead of four keeps the kernel's code in the instruction
        // cache
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            load(ks, 0);
#pragma unroll
            for (int i = 0; i < KPW; ++i)
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    if (u > 0 && !r2) continue;
                    const double aw = (double)av[0][u] * (double)w[0][i];
                    acc[i][u][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aw, (double)bv[0][0], acc[i][u][0], 0, 0, 0);
                    if (NV > 1 && c2)
                        acc[i][u][NV - 1] =
                            __builtin_amdgcn_mfma_f64_16x16x4f64(aw, (double)bv[0][NV - 1], acc[i][u][NV - 1], 0, 0, 0);
                }
        }
    } else {
        // FP32: k-steps in pairs, buffer 0 holding the even step and buffer 1
        // the odd one (NKS is even), the next step's operands read while the
        // current step's MFMAs issue
        flt4 c32[KPW][NA][NV];
#pragma unroll
        for (int i = 0; i < KPW; ++i)
#pragma unroll
            for (int u = 0; u < NA; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) c32[i][u][v] = flt4{0.f, 0.f, 0.f, 0.f};
        auto step = [&](int b) {
#pragma unroll
            for (int i = 0; i < KPW; ++i)
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    const float aw = (float)av[b][u] * (float)w[b][i];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        c32[i][u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw, (float)bv[b][v], c32[i][u][v], 0, 0, 0);
                }
            __builtin_amdgcn_sched_barrier(0);
        };
        load(0, 0);
#pragma unroll 1
        for (int ks = 0; ks < NKS; ks += 2) {
            load(ks + 1, 1);
            step(0);
            if (ks + 2 < NKS) load(ks + 2, 0);
            step(1);
        }
        // chunk sums into the FP64 accumulators (register r keeps the FP32 layout)
#pragma unroll
        for (int i = 0; i < KPW; ++i)
#pragma unroll
            for (int u = 0; u < NA; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][u][v][r] += (double)c32[i][u][v][r];
    }
}

// NA, NV: active row halves (of the wave's NMT) and column halves of the
// tile, fixed per workgroup: subtiles wholly outside the block are left out
// at compile time.  SPW = 2: NA = 1 for every wave, and a wave whose row
// half lies outside the block skips its MFMAs (one branch per chunk).
template <bool MIXED, int KPW, int SPW, int NA, int NV>
__device__ void contract_tile(const ContractArgs& a, int y, int piece, int s, int t, int a0, int b0, bool r2, bool c2,
                              bool upper, ContractLds<typename std::conditional<MIXED, float, double>::type,
                                                      contract_chunk<MIXED>()>& L) {
    typedef typename std::conditional<MIXED, float, double>::type T;
    constexpr int NC = contract_chunk<MIXED>();   // nodes per chunk
    constexpr int NPT = NC / 8;                   // nodes per loader thread and row
    auto& As = L.As;
    auto& Bs = L.Bs;
    auto& fl = L.fl;
    auto& wk = L.wk;
    const Meta2C& m = *a.m;
    // weights of this block (st_nw) and of this tile: all of them, or the
    // target potential alone (weight 1) above the diagonal of a block (s, s)
    // whose overlap follows from the transposed tile (overlap_mirrored)
    const int n_w = upper ? 1 : st_nw(m.same, m.n_w, s, t), w0 = upper ? 1 : 0;
    const int nk = st_nk(s, t, n_w);
    const int o1 = abs(s - t), o2 = s + t;
    const int nA = m.nA[s], nB = m.nB[t];
    const size_t nn = m.n_nodes;
    const double* nd = a.nodes + (size_t)y * m.n_fields * nn;
    // this work item's node range [p_begin, p_end) (whole chunks)
    const int nact_all = a.n_act[y];
    const int span = ((nact_all + m.n_split - 1) / m.n_split + NC - 1) / NC * NC;
    const int p_begin = piece * span;
    const int nact = min(nact_all, p_begin + span);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // loader roles: row (column) lr of A (B), NPT consecutive nodes from kq;
    // up to two node fields of the weights per thread (field ffi + q * 256 / NC)
    const int lr = tid >> 3, kq = (tid & 7) * NPT;
    const bool okA = a0 + lr < nA, okB = b0 + lr < nB;
    const T* arow = reinterpret_cast<const T*>(a.AT) + ((size_t)y * m.rowsT + m.rowT_off[s] + a0 + (okA ? lr : 0)) * nn;
    const T* brow = reinterpret_cast<const T*>(a.BT) + ((size_t)y * m.rowsP + m.rowP_off[t] + b0 + (okB ? lr : 0)) * nn;
    const int ffi = tid / NC, fk = tid % NC;
    constexpr int kFStep = kStageThreads2C / NC;
    int fid[2] = {0, 0};
    {
        const int ids[kWFields] = {kFCos, kFSin, kFW, kFW + 1, kFW + 2, kFJ + o1, kFJ + o2};
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (ffi + q * kFStep < kWFields) fid[q] = ids[ffi + q * kFStep];
    }
    // weight roles: node fk, weights kk = ffi + q * kFStep (q < kWIt) as the
    // fl rows of its three factors (Bessel order, cos/sin, quadrature weight)
    // packed in 4-bit fields, -1 past nk
    constexpr int kWIt = (NC * kMaxK + kStageThreads2C - 1) / kStageThreads2C;
    int wsel[kWIt];
#pragma unroll
    for (int q = 0; q < kWIt; ++q) {
        const int kk = ffi + q * kFStep;
        const int order = kk / (2 * n_w), trig = (kk / n_w) & 1, w = kk % n_w;
        wsel[q] = kk < nk ? (5 + order) | (trig << 4) | ((2 + w0 + w) << 8) : -1;
    }
    // this wave's weights and subtiles
    const int kk0 = SPW == 4 ? wave * KPW : (wave & 1) * KPW;
    const int mt0 = SPW == 4 ? 0 : (wave >> 1);
    constexpr int NMT = SPW == 4 ? 2 : 1;   // row halves covered by the wave
    const int li = lane & 15, lk = lane >> 4;
    // SPW = 2: whether the wave's row half lies inside the block (wave-uniform)
    const bool rows_in = SPW == 4 || a0 + mt0 * 16 < nA;

    T ra[NPT], rb[NPT];
    double rf[2] = {0.0, 0.0};
    auto fetch = [&](int base) {
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            const int p = base + kq + e;
            ra[e] = (okA && p < nact) ? arow[p] : (T)0;
            rb[e] = (okB && p < nact) ? brow[p] : (T)0;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (ffi + q * kFStep < kWFields) rf[q] = (base + fk < nact) ? nd[(size_t)fid[q] * nn + base + fk] : 0.0;
    };

    dbl4 acc[KPW][NMT][2];
#pragma unroll
    for (int i = 0; i < KPW; ++i)
#pragma unroll
        for (int u = 0; u < NMT; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) acc[i][u][v] = dbl4{0.0, 0.0, 0.0, 0.0};

    if (p_begin < nact) fetch(p_begin);
    for (int base = p_begin; base < nact; base += NC) {
#pragma unroll
        for (int e = 0; e < NPT; ++e) {
            As[kq + e][lr ^ lds_swz(kq + e)] = ra[e];
            Bs[kq + e][lr ^ lds_swz(kq + e)] = rb[e];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (ffi + q * kFStep < kWFields) fl[ffi + q * kFStep][fk] = rf[q];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kWIt; ++q)
            if (wsel[q] >= 0)
                wk[fk][ffi + q * kFStep] = fl[wsel[q] & 15][fk] * fl[(wsel[q] >> 4) & 15][fk] * fl[wsel[q] >> 8][fk];
        __syncthreads();
        // next chunk's operands in flight during this chunk's MFMA
        if (base + NC < nact) fetch(base + NC);
        if (rows_in) chunk_mfma<MIXED, KPW, NMT, NA, NV>(L, mt0, kk0, li, lk, r2, c2, acc);
        __syncthreads();
    }
    double* out = a.tmol + ((size_t)y * m.n_split + piece) * m.n_tmol + m.st_off[s][t];
#pragma unroll
    for (int i = 0; i < KPW; ++i) {
        const int kk = kk0 + i;
        // position of weight kk of the tile in the block's (order, trig, weight)
        // layout: an upper tile's weight kk is the target potential (weight 1
        // of the block's two) of (order, trig) = kk
        const int ko = upper ? 2 * kk + 1 : kk;
#pragma unroll
        for (int u = 0; u < NA; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int jj = b0 + v * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ii = a0 + (mt0 + u) * 16 + (MIXED ? mfma_row_f32(r, lane) : mfma_row_f64(r, lane));
                    if (kk < nk && ii < nA && jj < nB) out[((size_t)ko * nA + ii) * nB + jj] = acc[i][u][v][r];
                }
            }
    }
}

// One workgroup per (job, tile) with an XCD-aware order: consecutive
// workgroup ids go to the eight XCDs in turn, and the work items of XCD x are
// the x-th eighth of the job-major list, so the tiles of one job (which
// stream the same operand rows) share an L2.  Per chunk of nodes (32, or 64
// for the FP32 products) the 32 rows of A, the 32 columns of B and the node
// fields of the weights are loaded into registers one chunk ahead (their latency overlaps the MFMA
// of the current chunk), then staged in LDS; the waves split the nk weights
// and the four 16 x 16 subtiles as contract_tile describes and feed the MFMA
// with (A w_k) and B.
//
// MIXED: the products run on v_mfma_f32_16x16x4f32 (operands in FP32,
// accumulated in FP32 over the 64 nodes of a chunk) and each chunk's partial
// sums are added to FP64 accumulators, so the FP32 accumulation error stays
// that of a 64-term sum whatever the number of nodes.
template <bool MIXED>
__global__ __launch_bounds__(kStageThreads2C, MIXED ? 2 : 3) void k_2c_contract(ContractArgs a) {
    const Meta2C& m = *a.m;
    const int per_job = m.n_tiles * m.n_split;
    const int total = per_job * a.n_jobs;
    const int per = (total + 7) / 8;
    const int W = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (W >= total) return;
    const int y = W / per_job;
    const int rem = W - y * per_job;
    const int piece = rem / m.n_tiles;
    const int2 tl = a.tiles[rem - piece * m.n_tiles];
    const int s = tl.x & 0xff, t = (tl.x >> 8) & 0xff, a0 = tl.y & 0xffff, b0 = tl.y >> 16;
    const bool upper = (tl.x & kTileUpper) != 0;
    __shared__ ContractLds<typename std::conditional<MIXED, float, double>::type, contract_chunk<MIXED>()> L;
    // second row / column half of the 32 x 32 tile inside the block
    const bool r2 = a0 + 16 < m.nA[s], c2 = b0 + 16 < m.nB[t];
    // FP32 products: one compiled variant per set of active subtiles; FP64:
    // one variant that tests r2 and c2 at run time
#define WPCCC_TILE4(KPW)                                                                          \
    if (!MIXED || (r2 && c2)) contract_tile<MIXED, KPW, 4, 2, 2>(a, y, piece, s, t, a0, b0, r2, c2, upper, L); \
    else if (r2) contract_tile<MIXED, KPW, 4, 2, 1>(a, y, piece, s, t, a0, b0, r2, c2, upper, L);              \
    else if (c2) contract_tile<MIXED, KPW, 4, 1, 2>(a, y, piece, s, t, a0, b0, r2, c2, upper, L);              \
    else contract_tile<MIXED, KPW, 4, 1, 1>(a, y, piece, s, t, a0, b0, r2, c2, upper, L);
#define WPCCC_TILE2(KPW)                                                                          \
    if (!MIXED || c2) contract_tile<MIXED, KPW, 2, 1, 2>(a, y, piece, s, t, a0, b0, r2, c2, upper, L);         \
    else contract_tile<MIXED, KPW, 2, 1, 1>(a, y, piece, s, t, a0, b0, r2, c2, upper, L);
    switch (st_nk(s, t, upper ? 1 : st_nw(m.same, m.n_w, s, t))) {
        case 2: WPCCC_TILE2(1) break;
        case 4: WPCCC_TILE4(1) break;
        case 6: WPCCC_TILE2(3) break;
        case 8: WPCCC_TILE4(2) break;
        default: WPCCC_TILE4(3) break;
    }
#undef WPCCC_TILE4
#undef WPCCC_TILE2
}

// Sum of the node-range partial sums of the contraction into range 0, in
// range order: tmol[job][0][e] = ((T_0 + T_1) + T_2) + ...; grid: x over
// n_tmol / 256, y = job.
__global__ __launch_bounds__(256) void k_2c_reduce(double* __restrict__ tmol, int n_tmol, int n_split) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_tmol) return;
    double* t = tmol + (size_t)blockIdx.y * n_split * n_tmol + e;
    double acc = t[0];
    for (int q = 1; q < n_split; ++q) acc += t[(size_t)q * n_tmol];
    t[0] = acc;
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
    const double* tm = a.tmol + (size_t)blockIdx.y * m.n_split * m.n_tmol;
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
            const int nwb = st_nw(m.same, n_w, s, t);
            if (nwb) {
                const size_t blk = (size_t)m.nA[s] * nBt;
                const double* base = tm + m.st_off[s][t] + (size_t)is * nBt + jt;
                // above the diagonal of a block (s, s) the overlap is that of
                // (b, a) under the same exchange map (overlap_mirrored)
                const bool ovl_t = overlap_mirrored(m.same, s, t, is, jt);
                const double* bt = tm + m.st_off[s][t] + (size_t)jt * nBt + is;
                const double sgt = ((la + lb) & 1) ? -1.0 : 1.0;
                for (int w = 0; w < n_w; ++w) {
                    double tc, ts;
                    if (w == 0 && ovl_t) {
                        tc = sgt * bt[(size_t)((order * 2 + 0) * nwb) * blk];
                        ts = -sgt * bt[(size_t)((order * 2 + 1) * nwb) * blk];
                    } else {
                        tc = base[(size_t)((order * 2 + 0) * nwb + w) * blk];
                        ts = base[(size_t)((order * 2 + 1) * nwb + w) * blk];
                    }
                    acc[w][0] += c * (pr * tc - pi * ts);
                    acc[w][1] += c * (pr * ts + pi * tc);
                }
            } else {
                // one basis on both centres, s > t: tau -> -tau exchanges the
                // centres, so T_(s,t),W[a][b] = (-1)^(l_a+s+l_b+t) (+cos, -sin)
                // T_(t,s),W'[b][a] with W' = W for the overlap and the
                // projectile potential for the target potential
                const int nw2 = st_nw(m.same, n_w, t, s);
                const size_t blk2 = (size_t)m.nA[t] * m.nB[s];
                const double* base2 = tm + m.st_off[t][s] + (size_t)jt * m.nB[s] + is;
                const double sg = ((la + s + lb + t) & 1) ? -1.0 : 1.0;
                for (int w = 0; w < n_w; ++w) {
                    const int w2 = w == 0 ? 0 : 2;
                    const double tc = sg * base2[(size_t)((order * 2 + 0) * nw2 + w2) * blk2];
                    const double ts = -sg * base2[(size_t)((order * 2 + 1) * nw2 + w2) * blk2];
                    acc[w][0] += c * (pr * tc - pi * ts);
                    acc[w][1] += c * (pr * ts + pi * tc);
                }
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
    if (m.mirror) {
        // one basis on both centres: tau -> -tau exchanges the centres, turns
        // the target potential's weight into the projectile's and conjugates
        // the translation phase, so the prior block's element at (projectile
        // state al, target state be) is (-1)^(l_a + l_b) Q_(al, be)
        const double sg = ((la + lb) & 1) ? -1.0 : 1.0;
        H[(size_t)(NT + al) * N + be] = make_double2(sg * val[1].x, sg * val[1].y);
    } else {
        const double2 low = (m.q_prior && n_w > 2) ? val[2] : val[1];
        H[(size_t)col * N + row] = make_double2(low.x, -low.y);     // Q^dagger or the prior form
    }
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

// y = P (H u) (or y = M u) for every path of the launch: grid x = blocks of 16 rows,
// y = path; each wave accumulates four rows at once (four 1 KB row segments
// in flight per iteration).
__global__ __launch_bounds__(256) void k_2c_hu(Stage2CArgs a) {
    const PathMats pm = a.pm[blockIdx.y];
    const int j = pm.path, N = pm.N;
    if ((int)blockIdx.x * 16 >= N) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double2* H = pm.H + (size_t)a.slot * N * N;
    const int* perm = pm.perm ? pm.perm + (size_t)a.slot * N : nullptr;
    const double2* u = a.u_in + (size_t)j * a.n_pad;
    const int r0 = blockIdx.x * 16 + wave * 4;
    const double2* hr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = min(r0 + q, N - 1);
        hr[q] = H + (size_t)(perm ? perm[row] : row) * N;
    }
    double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = lane; c < N; c += 64) {
        const double2 x = u[c];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 h = hr[q][c];
            re[q] += h.x * x.x - h.y * x.y;
            im[q] += h.x * x.y + h.y * x.x;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int off = 32; off > 0; off >>= 1) {
            re[q] += __shfl_xor(re[q], off, 64);
            im[q] += __shfl_xor(im[q], off, 64);
        }
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (r0 + q < N) a.Y[(size_t)j * a.n_pad + r0 + q] = make_double2(re[q], im[q]);
}

constexpr int kSolveBlock = 32;
// threads of a k_2c_solve workgroup (one per path): the block updates are
// matrix-vector products over up to N rows, so more threads keep more LU
// loads in flight on the path's CU
constexpr int kSolveThreads = 1024;

// y <- U^{-1} L^{-1} y (where the stage solves), K = -(i/v) y and the RK4
// update; one workgroup per path.  The triangular solves go by blocks of 32 rows: the diagonal block is
// staged in LDS and solved by one wave with lane shuffles, then all waves
// update the rows below (above) it from the column-major factors.
__global__ __launch_bounds__(kSolveThreads) void k_2c_solve(Stage2CArgs a) {
    extern __shared__ double2 ys[];      // [N]
    __shared__ double2 blk[kSolveBlock][kSolveBlock + 1];
    const PathMats pm = a.pm[blockIdx.x];
    const int j = pm.path, N = pm.N, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const double2* LU = pm.LU + (size_t)a.slot * N * N;
    for (int i = tid; i < N; i += blockDim.x) ys[i] = a.Y[(size_t)j * a.n_pad + i];
    __syncthreads();
    // L (unit diagonal): forward
    for (int kb = 0; a.solve && kb < N; kb += kSolveBlock) {
        const int nbk = min(kSolveBlock, N - kb);
        for (int e = tid; e < nbk * nbk; e += blockDim.x) {
            const int r = e % nbk, c = e / nbk;
            blk[r][c] = LU[(kb + r) + (size_t)(kb + c) * N];
        }
        __syncthreads();
        if (wave == 0) {
            double2 y = (lane < nbk) ? ys[kb + lane] : make_double2(0.0, 0.0);
            for (int c = 0; c + 1 < nbk; ++c) {
                const double yr = __shfl(y.x, c, 64), yi = __shfl(y.y, c, 64);
                if (lane > c && lane < nbk) {
                    const double2 l = blk[lane][c];
                    y.x -= l.x * yr - l.y * yi;
                    y.y -= l.x * yi + l.y * yr;
                }
            }
            if (lane < nbk) ys[kb + lane] = y;
        }
        __syncthreads();
        for (int i = kb + nbk + tid; i < N; i += blockDim.x) {
            double re = 0.0, im = 0.0;
#pragma unroll 8
            for (int c = 0; c < nbk; ++c) {
                const double2 l = LU[i + (size_t)(kb + c) * N], x = ys[kb + c];
                re += l.x * x.x - l.y * x.y;
                im += l.x * x.y + l.y * x.x;
            }
            ys[i].x -= re;
            ys[i].y -= im;
        }
        __syncthreads();
    }
    // U: backward
    for (int kb = ((N - 1) / kSolveBlock) * kSolveBlock; a.solve && kb >= 0; kb -= kSolveBlock) {
        const int nbk = min(kSolveBlock, N - kb);
        for (int e = tid; e < nbk * nbk; e += blockDim.x) {
            const int r = e % nbk, c = e / nbk;
            blk[r][c] = LU[(kb + r) + (size_t)(kb + c) * N];
        }
        __syncthreads();
        if (wave == 0) {
            double2 y = (lane < nbk) ? ys[kb + lane] : make_double2(0.0, 0.0);
            for (int c = nbk - 1; c >= 0; --c) {
                if (lane == c) {
                    const double2 d = blk[c][c];
                    const double dn = d.x * d.x + d.y * d.y;
                    y = make_double2((y.x * d.x + y.y * d.y) / dn, (y.y * d.x - y.x * d.y) / dn);
                }
                const double yr = __shfl(y.x, c, 64), yi = __shfl(y.y, c, 64);
                if (lane < c) {
                    const double2 uu = blk[lane][c];
                    y.x -= uu.x * yr - uu.y * yi;
                    y.y -= uu.x * yi + uu.y * yr;
                }
            }
            if (lane < nbk) ys[kb + lane] = y;
        }
        __syncthreads();
        for (int i = tid; i < kb; i += blockDim.x) {
            double re = 0.0, im = 0.0;
#pragma unroll 8
            for (int c = 0; c < nbk; ++c) {
                const double2 uu = LU[i + (size_t)(kb + c) * N], x = ys[kb + c];
                re += uu.x * x.x - uu.y * x.y;
                im += uu.x * x.y + uu.y * x.x;
            }
            ys[i].x -= re;
            ys[i].y -= im;
        }
        __syncthreads();
    }
    const double sc = 1.0 / a.vvec[j];
    const double h = a.hdev ? a.hdev[3 * (size_t)(*a.step) + 2] : a.h;
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

// dK[r][c] = (S_+[r][N_T + c] - S_-[r][N_T + c]) / (2 dz): the K block of the
// central difference of S (its identity blocks do not vary)
__global__ __launch_bounds__(256) void k_2c_dk(SymArgs a) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.NT * a.NP) return;
    const int pl = a.path0 + blockIdx.y, r = e / a.NP, c = e % a.NP;
    const size_t NN = (size_t)a.N * a.N, at = r + (size_t)(a.NT + c) * a.N;
    const double2 sp = a.S[((size_t)pl * kSlots2C + a.slot_p) * NN + at];
    const double2 sm = a.S[((size_t)pl * kSlots2C + a.slot_m) * NN + at];
    a.dK[((size_t)pl * 2 + a.which) * a.NT * a.NP + e] =
        make_double2((sp.x - sm.x) * a.inv_2dz, (sp.y - sm.y) * a.inv_2dz);
}

// H <- (H + H^dag)/2 - (i v / 2) dS/dz in place, dS/dz = [[0, dK], [dK^dag, 0]]:
// each thread owns one unordered pair (r, c), r <= c, and writes both
// elements.  Grid x: 16 x 16 blocks of the upper triangle (lower blocks
// exit), y: paths.
__global__ __launch_bounds__(256) void k_2c_symm(SymArgs a) {
    const int nb = (a.N + 15) / 16;
    const int br = blockIdx.x / nb, bc = blockIdx.x % nb;
    if (br > bc) return;
    const int r = br * 16 + (threadIdx.x >> 4), c = bc * 16 + (threadIdx.x & 15);
    if (r > c || c >= a.N) return;
    const int pl = a.path0 + blockIdx.y;
    const double hv = 0.5 * a.vvec[a.paths[pl]];
    double2* H = a.H + ((size_t)pl * kSlots2C + a.slot) * (size_t)a.N * a.N;
    const double2 hrc = H[(size_t)r * a.N + c], hcr = H[(size_t)c * a.N + r];
    double2 d = make_double2(0.0, 0.0);  // dS/dz at (r, c)
    if (r < a.NT && c >= a.NT) d = a.dK[((size_t)pl * 2 + a.which) * a.NT * a.NP + (size_t)r * a.NP + (c - a.NT)];
    // (H + H^dag)/2 at (r, c) and (c, r); -(i v/2) d = (v/2) (d.y, -d.x); at (c, r) d -> conj(d)
    const double2 m = make_double2(0.5 * (hrc.x + hcr.x), 0.5 * (hrc.y - hcr.y));
    if (r == c) {
        H[(size_t)r * a.N + c] = make_double2(m.x, 0.0);
        return;
    }
    H[(size_t)r * a.N + c] = make_double2(m.x + hv * d.y, m.y - hv * d.x);
    H[(size_t)c * a.N + r] = make_double2(m.x - hv * d.y, -m.y - hv * d.x);
}

__global__ void k_transpose_copy(const double2* __restrict__ src, double2* __restrict__ dst, int N) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c < N) dst[(size_t)r * N + c] = src[r + (size_t)c * N];
}

}  // namespace

hipError_t launch_2c_nodes(const NodeArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_2c_nodes, dim3((hm.n_nodes + 255) / 256, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Dynamic LDS of k_2c_interp: the larger of the stencil weights (64 x 5) and
// the Legendre factors of the widest l range of a 64-function tile.
size_t interp_lds_bytes(const Meta2C& hm) {
    int npf = 5;
    for (int side = 0; side < 2; ++side) {
        const int nf = side ? hm.nfP : hm.nfT, ls = side ? hm.LP : hm.LT;
        const int* rad_off = side ? hm.radP_off : hm.radT_off;
        for (int f0 = 0; f0 < nf; f0 += 64) {
            const int fend = std::min(f0 + 64, nf);
            int l_lo = 0, l_hi = 0;
            while (l_lo < ls && rad_off[l_lo + 1] <= f0) ++l_lo;
            while (l_hi < ls && rad_off[l_hi + 1] <= fend - 1) ++l_hi;
            npf = std::max(npf, (l_hi + 1) * (l_hi + 2) / 2 - l_lo * (l_lo + 1) / 2);
        }
    }
    return (size_t)npf * 64 * sizeof(double);
}

hipError_t launch_2c_interp(const InterpArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const dim3 grid((hm.n_nodes + 63) / 64, (hm.nfT + 63) / 64 + (hm.nfP + 63) / 64, n_jobs), block(256);
    const size_t smem = interp_lds_bytes(hm);
    // above 64 KiB per workgroup (the factors of a tile that spans many l)
    // the kernels need the larger limit, set once (thread-safe static
    // initialisation) to a fixed value that no later call lowers
    static const hipError_t raised = [] {
        hipError_t e = hipSuccess;
        for (const void* f : {(const void*)k_2c_interp<float>, (const void*)k_2c_interp<double>})
            if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kInterpMaxDynLds);
        return e;
    }();
    if (raised != hipSuccess) return raised;
    if (hm.mixed)
        WPCCC_LAUNCH(ev, k_2c_interp<float>, grid, block, smem, st, a);
    else
        WPCCC_LAUNCH(ev, k_2c_interp<double>, grid, block, smem, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_contract(const ContractArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const dim3 grid(8 * ((hm.n_tiles * hm.n_split * n_jobs + 7) / 8)), block(kStageThreads2C);
    if (hm.mixed)
        WPCCC_LAUNCH(ev, k_2c_contract<true>, grid, block, 0, st, a);
    else
        WPCCC_LAUNCH(ev, k_2c_contract<false>, grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_reduce(double* tmol, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    if (hm.n_split < 2) return hipSuccess;
    WPCCC_LAUNCH(ev, k_2c_reduce, dim3((hm.n_tmol + 255) / 256, n_jobs), dim3(256), 0, st, tmol, hm.n_tmol, hm.n_split);
    return hipGetLastError();
}

hipError_t launch_2c_assemble(const AssembleArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const int nb = (hm.NT * hm.NP + 255) / 256 + (hm.NT * hm.NT + hm.NP * hm.NP + 255) / 256;
    WPCCC_LAUNCH(ev, k_2c_assemble, dim3(nb, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_setup_batch(const SetupBatchArgs& a, const Meta& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const int nbG = (hm.n_g + 255) / 256;
    WPCCC_LAUNCH(ev, k_setup_batch, dim3(a.nbF + a.nbP + nbG, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_direct(const DirectArgs& a, const Meta2C& hm, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const int nb = (hm.NT * hm.NT + hm.NP * hm.NP + 255) / 256;
    WPCCC_LAUNCH(ev, k_2c_direct, dim3(nb, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_hu(const Stage2CArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_2c_hu, dim3((a.N_max + 15) / 16, n_paths), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_solve(const Stage2CArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_2c_solve, dim3(n_paths), dim3(kSolveThreads), a.N_max * sizeof(double2), st, a);
    return hipGetLastError();
}

hipError_t launch_2c_finish(const double2* X, const double2* S, int N, int n_pad, const int* paths, int n_paths,
                            int slot, double* P, double* norm, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_2c_finish, dim3(n_paths), dim3(256), 0, st, X, S, N, n_pad, paths, slot, P, norm);
    return hipGetLastError();
}

hipError_t launch_transpose_copy(const double2* src, double2* dst, int N, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_copy, dim3((N + 255) / 256, N), dim3(256), 0, st, src, dst, N);
    return hipGetLastError();
}

}  // namespace wpccc

// ---------------------------------------------------------------------------
// Sustained matrix-core rate: every wave issues iters x 8 independent MFMAs
// (eight accumulators, so no MFMA waits for another's result).
namespace wpccc {
namespace {

template <bool F64>
__global__ __launch_bounds__(256) void k_mfma_rate(double* out, int iters) {
    const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
    double s = 0.0;
    if (F64) {
        dbl4 acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = dbl4{0.0, 0.0, 0.0, 0.0};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    } else {
        flt4 acc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) acc[i] = flt4{0.f, 0.f, 0.f, 0.f};
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int i = 0; i < 8; ++i)
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, acc[i], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;   // keeps the products live
}

}  // namespace

hipError_t measure_mfma(double* tf64, double* tf32, hipStream_t st) {
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const int grid = 4 * n_cu, iters = 8000;
    double* out = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipMalloc(&out, (size_t)grid * 256 * sizeof(double));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const double flops = (double)grid * 4 * iters * 8 * 2048.0;  // 4 waves, 8 MFMAs of 16 x 16 x 4 x 2
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        for (int f64 = 1; f64 >= 0 && e == hipSuccess; --f64) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) {
                if (f64)
                    hipLaunchKernelGGL(k_mfma_rate<true>, dim3(grid), dim3(256), 0, st, out, iters);
                else
                    hipLaunchKernelGGL(k_mfma_rate<false>, dim3(grid), dim3(256), 0, st, out, iters);
                e = hipGetLastError();
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && pass == 1) {   // pass 0 warms the clocks
                double* dst = f64 ? tf64 : tf32;
                if (dst) *dst = flops / ((double)ms * 1e-3) / 1e12;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out) (void)hipFree(out);
    return e;
}

hipError_t launch_2c_dk(const SymArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_2c_dk, dim3((a.NT * a.NP + 255) / 256, n_paths), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_2c_symm(const SymArgs& a, int n_paths, hipStream_t st, const LaunchEv& ev) {
    const int nb = (a.N + 15) / 16;
    WPCCC_LAUNCH(ev, k_2c_symm, dim3(nb * nb, n_paths), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace wpccc

// Batched complex LU with partial pivoting (the overlap matrices S of Eq. 1)
// on gfx950.  Right-looking, one panel of kLUPanel columns per pass and one
// launch of each kernel per pass for every matrix of the batch:
//   k_lu_panel      the N - k0 rows of the panel in registers (one to four
//                   rows per thread, 512 threads): per column an argmax (largest
//                   |a|^2, ties to the lowest row), the row swap, the scaling
//                   of L and the rank-1 update of the remaining panel columns
//   k_lu_swap_trsm  the panel's swaps on every other column (LAPACK getrf
//                   order) and U12 = L11^-1 A12, one thread per column
//   k_lu_update     A22 -= L21 U12 on MFMA (v_mfma_f64_16x16x4f64), 64 x 64
//                   output tiles, complex product as four real products
// and, for the explicit form of the derivative matrix, k_lu_rhs: M = S^-1 H
// from the finished factors.
#include <hip/hip_runtime.h>

#include "plan2c.h"

namespace wpccc {

namespace {

constexpr int kPanelThreads = 512;

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline void job_of(const Jobs& J, int y, int& pl, int& slot) {
    pl = J.path0 + y / J.n_sub;
    slot = J.slot[y % J.n_sub];
}

// Whether a launch's kernel has nothing to do for this matrix (LUStepArgs::skip_mode).
__device__ inline bool skipped(const LUStepArgs& a, size_t ms) {
    if (a.skip_mode == 0) return false;
    const bool s = a.skip[ms] != 0;
    return a.skip_mode == 1 ? s : !s;
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ROWS rows per thread (N - k0 <= ROWS x 512), panels of up to NB columns: the
// panel's N - k0 rows live in registers (ROWS x NB complex values per thread).
template <int ROWS, int NB>
__global__ __launch_bounds__(kPanelThreads) void k_lu_panel(LUStepArgs a) {
    constexpr int kPanelRows = ROWS;
    __shared__ double2 prow[NB], xrow[NB];
    __shared__ double redv[kPanelThreads / 64];
    __shared__ int redi[kPanelThreads / 64];
    int pl, slot;
    job_of(a.jobs, blockIdx.x, pl, slot);
    const int N = a.N, k0 = a.k0, nb = a.nb;
    const size_t ms = (size_t)pl * kSlots2C + slot;
    if (skipped(a, ms)) return;
    double2* A = a.LU + ms * (size_t)N * N;
    int* piv = a.piv + ms * N;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (k0 == 0) {
        int* perm = a.perm + ms * N;
        for (int i = t; i < N; i += kPanelThreads) perm[i] = i;
    }
    double2 v[kPanelRows][NB];
#pragma unroll
    for (int q = 0; q < kPanelRows; ++q) {
        const int i = k0 + t + kPanelThreads * q;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            v[q][c] = (i < N && c < nb) ? A[i + (size_t)(k0 + c) * N] : make_double2(0.0, 0.0);
    }
#pragma clang loop unroll(full)
    for (int jj = 0; jj < NB; ++jj) {
        if (jj < nb) {
        const int j = k0 + jj;
        double best = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < kPanelRows; ++q) {
            const int i = k0 + t + kPanelThreads * q;
            const double m = v[q][jj].x * v[q][jj].x + v[q][jj].y * v[q][jj].y;
            if (i >= j && i < N && m > best) {
                best = m;
                bi = i;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (lane == 0) {
            redv[wave] = best;
            redi[wave] = bi;
        }
        __syncthreads();
        double pmag = redv[0];
        int p = redi[0];
        for (int w = 1; w < kPanelThreads / 64; ++w)
            if (redv[w] > pmag || (redv[w] == pmag && redi[w] < p)) {
                pmag = redv[w];
                p = redi[w];
            }
        if (!(pmag > 0.0)) {
            // exact zero column: record, leave it (LAPACK continues the same way)
            if (t == 0) {
                piv[j] = j;
                if (atomicCAS(&a.flag[1], 0, a.paths[pl] + 1) == 0) a.flag[2] = j;
            }
        } else {
        if (t == 0) piv[j] = p;
        const int oj = (j - k0) % kPanelThreads, qj = (j - k0) / kPanelThreads;
        const int op = (p - k0) % kPanelThreads, qp = (p - k0) / kPanelThreads;
#pragma unroll
        for (int q = 0; q < kPanelRows; ++q) {
            if (t == op && q == qp)
#pragma unroll
                for (int c = 0; c < NB; ++c) prow[c] = v[q][c];
            if (t == oj && q == qj && p != j)
#pragma unroll
                for (int c = 0; c < NB; ++c) xrow[c] = v[q][c];
        }
        __syncthreads();
        if (p != j) {
#pragma unroll
            for (int q = 0; q < kPanelRows; ++q) {
                if (t == oj && q == qj)
#pragma unroll
                    for (int c = 0; c < NB; ++c) v[q][c] = prow[c];
                if (t == op && q == qp)
#pragma unroll
                    for (int c = 0; c < NB; ++c) v[q][c] = xrow[c];
            }
        }
        const double2 d = prow[jj];
        const double dn = d.x * d.x + d.y * d.y;
        const double2 inv = make_double2(d.x / dn, -d.y / dn);
#pragma unroll
        for (int q = 0; q < kPanelRows; ++q) {
            const int i = k0 + t + kPanelThreads * q;
            if (i > j && i < N) {
                const double2 l = cmul(v[q][jj], inv);
                v[q][jj] = l;
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    if (c > jj) {
                        const double2 u = prow[c];
                        v[q][c].x -= l.x * u.x - l.y * u.y;
                        v[q][c].y -= l.x * u.y + l.y * u.x;
                    }
                }
            }
        }
        }
        __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < kPanelRows; ++q) {
        const int i = k0 + t + kPanelThreads * q;
        if (i < N)
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nb) A[i + (size_t)(k0 + c) * N] = v[q][c];
    }
}

// grid: x = column blocks of 256, y = matrix.
__global__ __launch_bounds__(256) void k_lu_swap_trsm(LUStepArgs a) {
    constexpr int NB = kLUPanel;
    __shared__ double2 L11[NB][NB];
    __shared__ int pv[NB];
    int pl, slot;
    job_of(a.jobs, blockIdx.y, pl, slot);
    const int N = a.N, k0 = a.k0, nb = a.nb;
    const size_t ms = (size_t)pl * kSlots2C + slot;
    if (skipped(a, ms)) return;
    double2* A = a.LU + ms * (size_t)N * N;
    const int* piv = a.piv + ms * N;
    const int t = threadIdx.x;
    for (int e = t; e < nb * nb; e += blockDim.x) {
        const int r = e % nb, c = e / nb;
        L11[r][c] = A[(k0 + r) + (size_t)(k0 + c) * N];
    }
    if (t < nb) pv[t] = piv[k0 + t];
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) {
        int* perm = a.perm + ms * N;
        for (int jj = 0; jj < nb; ++jj) {
            const int p = pv[jj];
            if (p != k0 + jj) {
                const int x = perm[k0 + jj];
                perm[k0 + jj] = perm[p];
                perm[p] = x;
            }
        }
    }
    const int c = blockIdx.x * blockDim.x + t;
    if (c >= N || (c >= k0 && c < k0 + nb)) return;
    double2* col = A + (size_t)c * N;
    for (int jj = 0; jj < nb; ++jj) {
        const int p = pv[jj];
        if (p != k0 + jj) {
            const double2 x = col[k0 + jj];
            col[k0 + jj] = col[p];
            col[p] = x;
        }
    }
    if (c < k0 + nb) return;
    double2 x[NB];
#pragma unroll
    for (int jj = 0; jj < NB; ++jj) x[jj] = (jj < nb) ? col[k0 + jj] : make_double2(0.0, 0.0);
#pragma unroll
    for (int jj = 1; jj < NB; ++jj) {
        if (jj < nb) {
#pragma unroll
            for (int m = 0; m < jj; ++m) {
                const double2 l = L11[jj][m];
                x[jj].x -= l.x * x[m].x - l.y * x[m].y;
                x[jj].y -= l.x * x[m].y + l.y * x[m].x;
            }
        }
    }
#pragma unroll
    for (int jj = 0; jj < NB; ++jj)
        if (jj < nb) col[k0 + jj] = x[jj];
}

// grid: x = 64 x 64 tiles of the trailing matrix (T x T), y = matrix.
// Computed as the transposed product D'[jj][ii] = sum_k U12[k][jj] L21[ii][k],
// so that the 16 lanes of an output row address consecutive rows of the
// column-major matrix.
__global__ __launch_bounds__(256) void k_lu_update(LUStepArgs a) {
    constexpr int NB = kLUPanel;
    __shared__ double Ur[NB][64], Ui[NB][64], Lr[NB][64], Li[NB][64];
    int pl, slot;
    job_of(a.jobs, blockIdx.y, pl, slot);
    const int N = a.N, k0 = a.k0, nb = a.nb, k1 = k0 + nb;
    const int T = (N - k1 + 63) / 64;
    const int bi = blockIdx.x % T, bj = blockIdx.x / T;
    const int r0 = k1 + 64 * bi, c0 = k1 + 64 * bj;
    const size_t ms = (size_t)pl * kSlots2C + slot;
    if (skipped(a, ms)) return;
    double2* A = a.LU + ms * (size_t)N * N;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int jsub = (wave >> 1) * 32, isub = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    dbl4 re[2][2], im[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            re[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
            im[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
    // the k range k0 .. k0 + nb - 1 in chunks of NB (one chunk for a panel)
    for (int kc = 0; kc < nb; kc += NB) {
    if (kc) __syncthreads();
    for (int e = t; e < 64 * NB; e += blockDim.x) {
        const int ii = e % 64, k = e / 64;
        const int row = r0 + ii;
        const double2 x = (row < N && kc + k < nb) ? A[row + (size_t)(k0 + kc + k) * N] : make_double2(0.0, 0.0);
        Lr[k][ii] = x.x;
        Li[k][ii] = x.y;
    }
    for (int e = t; e < 64 * NB; e += blockDim.x) {
        const int k = e % NB, jj = e / NB;
        const int col = c0 + jj;
        const double2 x = (col < N && kc + k < nb) ? A[(k0 + kc + k) + (size_t)col * N] : make_double2(0.0, 0.0);
        Ur[k][jj] = x.x;
        Ui[k][jj] = x.y;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < NB / 4; ++ks) {
        const int kr = ks * 4 + lk;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const double ur = Ur[kr][jsub + 16 * x + li], ui = Ui[kr][jsub + 16 * x + li];
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const double lr = Lr[kr][isub + 16 * y + li], lm = Li[kr][isub + 16 * y + li];
                re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ur, lr, re[x][y], 0, 0, 0);
                re[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ui, lm, re[x][y], 0, 0, 0);
                im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ur, lm, im[x][y], 0, 0, 0);
                im[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ui, lr, im[x][y], 0, 0, 0);
            }
        }
    }
    }
    // D'[row][col] of a 16 x 16 tile: lane l, register r -> row 4 r + l / 16, col l % 16
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = c0 + jsub + 16 * x + 4 * r + lk;
                const int row = r0 + isub + 16 * y + li;
                if (row < N && col < N) {
                    double2* p = A + row + (size_t)col * N;
                    double2 val = *p;
                    val.x -= re[x][y][r];
                    val.y -= im[x][y][r];
                    *p = val;
                }
            }
}

// One workgroup per matrix: skip = (every |A[i][j]| <= 1 for rows i >= nt,
// columns j < nt, i.e. |K^dagger| <= 1); where set, the identity permutation
// and the diagonal pivots of the first nt columns are written here (the panel
// steps that would write them return at once).
__global__ __launch_bounds__(1024) void k_lu_check(LUStepArgs a) {
    __shared__ int bad;
    int pl, slot;
    job_of(a.jobs, blockIdx.x, pl, slot);
    const int N = a.N, nt = a.nt;
    const size_t ms = (size_t)pl * kSlots2C + slot;
    const double2* A = a.LU + ms * (size_t)N * N;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    __syncthreads();
    // every element of the block independent of the others (all loads in
    // flight at once; consecutive threads read consecutive rows of a column)
    int b = 0;
    const int nr = N - nt;
    const long long n_el = (long long)nt * nr;
    for (long long e = t; e < n_el; e += blockDim.x) {
        const int j = (int)(e / nr), i = nt + (int)(e - (long long)j * nr);
        const double2 x = A[i + (size_t)j * N];
        b |= !(x.x * x.x + x.y * x.y <= 1.0);
    }
    if (b) atomicOr(&bad, 1);
    __syncthreads();
    const int ok = bad ? 0 : 1;
    if (t == 0) a.skip[ms] = ok;
    if (ok) {
        int* perm = a.perm + ms * N;
        int* piv = a.piv + ms * N;
        for (int i = t; i < N; i += blockDim.x) perm[i] = i;
        for (int j = t; j < nt; j += blockDim.x) piv[j] = j;
    }
}


// M = S^{-1} H = U^{-1} L^{-1} (P H) for every matrix of the launch from the
// factors above: the explicit form of Eq. INV, N right-hand sides.  One
// workgroup per (matrix, block of 32 columns of H).  Column blocks are
// independent, so a block's forward and backward substitutions run back to
// back in one workgroup, left-looking by blocks of 32 rows: a row block
// first subtracts its products with the finished blocks (32 x 32 tiles of
// the factor and of the solution staged in LDS; each thread holds one row
// and four columns), then solves its triangular diagonal block with
// shuffles across the 32 lanes that hold the block's rows.  The solution is
// written to M and read back by the later row blocks of the same workgroup.
constexpr int kRhsB = 32;

__global__ __launch_bounds__(256) void k_lu_rhs(RhsArgs a) {
    __shared__ double2 ft[kRhsB][kRhsB + 1];  // factor tile [row][k]
    __shared__ double2 yt[kRhsB][kRhsB + 1];  // right-hand-side / solution tile [row][column]
    const int N = a.N, t = threadIdx.x, r = t & 31, cq = (t >> 5) * 4;
    int pl, slot;
    job_of(a.jobs, blockIdx.y, pl, slot);
    const size_t ms = (size_t)pl * kSlots2C + slot, NN = (size_t)N * N;
    const double2* LU = a.LU + ms * NN;
    const int* perm = a.perm + ms * N;
    double2* M = a.M + ms * NN;
    const int c0 = blockIdx.x * kRhsB, nc = min(kRhsB, N - c0), nb = (N + kRhsB - 1) / kRhsB;
    const double2 zero = make_double2(0.0, 0.0);
    double2 acc[4];
    // rows [rb0, rb0 + 32) x columns [c0, c0 + 32) of a row-major matrix (row
    // i of the tile taken from row rows[rb0 + i] when rows is given), zero-padded
    auto load_rows = [&](const double2* src, const int* rows, int rb0) {
        for (int e = t; e < kRhsB * kRhsB; e += 256) {
            const int i = e >> 5, c = e & 31, row = rb0 + i;
            double2 v = zero;
            if (row < N && c < nc) v = src[(size_t)(rows ? rows[row] : row) * N + c0 + c];
            yt[i][c] = v;
        }
    };
    // rows [rb0, rb0 + 32) x columns [kb0, kb0 + 32) of the column-major factors, zero-padded
    auto load_factor = [&](int rb0, int kb0) {
        for (int e = t; e < kRhsB * kRhsB; e += 256) {
            const int i = e & 31, k = e >> 5, row = rb0 + i, col = kb0 + k;
            ft[i][k] = (row < N && col < N) ? LU[row + (size_t)col * N] : zero;
        }
    };
    auto subtract_products = [&]() {
#pragma unroll 8
        for (int k = 0; k < kRhsB; ++k) {
            const double2 f = ft[r][k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double2 y = yt[k][cq + q];
                acc[q].x -= f.x * y.x - f.y * y.y;
                acc[q].y -= f.x * y.y + f.y * y.x;
            }
        }
    };
    auto take_rows = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = yt[r][cq + q];
    };
    auto store_rows = [&](int rb0) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) yt[r][cq + q] = acc[q];
        __syncthreads();
        for (int e = t; e < kRhsB * kRhsB; e += 256) {
            const int i = e >> 5, c = e & 31, row = rb0 + i;
            if (row < N && c < nc) M[(size_t)row * N + c0 + c] = yt[i][c];
        }
    };
    // forward: L (unit diagonal) Y = P H
    for (int rb = 0; rb < nb; ++rb) {
        const int rb0 = rb * kRhsB;
        __syncthreads();
        load_rows(a.H + ms * NN, perm, rb0);
        __syncthreads();
        take_rows();
        for (int cb = 0; cb < rb; ++cb) {
            __syncthreads();
            load_factor(rb0, cb * kRhsB);
            load_rows(M, nullptr, cb * kRhsB);
            __syncthreads();
            subtract_products();
        }
        __syncthreads();
        load_factor(rb0, rb0);
        __syncthreads();
        for (int k = 0; k + 1 < kRhsB; ++k) {
            const double2 f = ft[r][k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double yr = __shfl(acc[q].x, k, 32), yi = __shfl(acc[q].y, k, 32);
                if (r > k) {
                    acc[q].x -= f.x * yr - f.y * yi;
                    acc[q].y -= f.x * yi + f.y * yr;
                }
            }
        }
        store_rows(rb0);
    }
    // backward: U M = Y
    for (int rb = nb - 1; rb >= 0; --rb) {
        const int rb0 = rb * kRhsB;
        __syncthreads();
        load_rows(M, nullptr, rb0);
        __syncthreads();
        take_rows();
        for (int cb = rb + 1; cb < nb; ++cb) {
            __syncthreads();
            load_factor(rb0, cb * kRhsB);
            load_rows(M, nullptr, cb * kRhsB);
            __syncthreads();
            subtract_products();
        }
        __syncthreads();
        load_factor(rb0, rb0);
        __syncthreads();
        for (int k = kRhsB - 1; k >= 0; --k) {
            if (r == k && rb0 + k < N) {
                const double2 d = ft[k][k];
                const double dn = d.x * d.x + d.y * d.y;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[q] = make_double2((acc[q].x * d.x + acc[q].y * d.y) / dn,
                                          (acc[q].y * d.x - acc[q].x * d.y) / dn);
            }
            const double2 f = ft[r][k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double yr = __shfl(acc[q].x, k, 32), yi = __shfl(acc[q].y, k, 32);
                if (r < k) {
                    acc[q].x -= f.x * yr - f.y * yi;
                    acc[q].y -= f.x * yi + f.y * yr;
                }
            }
        }
        store_rows(rb0);
    }
}

}  // namespace

hipError_t launch_lu_check(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_lu_check, dim3(n_jobs), dim3(1024), 0, st, a);
    return hipGetLastError();
}

int lu_panel_width(int N) { return N <= 2 * kPanelThreads ? kLUPanel : kLUPanel / 2; }

hipError_t launch_lu_panel(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    if (a.N > kLUMaxN || a.nb > lu_panel_width(a.N)) return hipErrorInvalidValue;
    // rows per thread from the rows left below k0 (the pivot is the same
    // whatever the split: largest |a|^2, lowest row on ties)
    const int rows = (a.N - a.k0 + kPanelThreads - 1) / kPanelThreads;
    if (lu_panel_width(a.N) == kLUPanel) {
        if (rows <= 1)
            WPCCC_LAUNCH(ev, (k_lu_panel<1, kLUPanel>), dim3(n_jobs), dim3(kPanelThreads), 0, st, a);
        else
            WPCCC_LAUNCH(ev, (k_lu_panel<2, kLUPanel>), dim3(n_jobs), dim3(kPanelThreads), 0, st, a);
    } else if (rows <= 1) {
        WPCCC_LAUNCH(ev, (k_lu_panel<1, kLUPanel / 2>), dim3(n_jobs), dim3(kPanelThreads), 0, st, a);
    } else if (rows <= 2) {
        WPCCC_LAUNCH(ev, (k_lu_panel<2, kLUPanel / 2>), dim3(n_jobs), dim3(kPanelThreads), 0, st, a);
    } else {
        WPCCC_LAUNCH(ev, (k_lu_panel<4, kLUPanel / 2>), dim3(n_jobs), dim3(kPanelThreads), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_lu_swap_trsm(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_lu_swap_trsm, dim3((a.N + 255) / 256, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lu_update(const LUStepArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    const int T = (a.N - a.k0 - a.nb + 63) / 64;
    if (T <= 0) return hipSuccess;
    WPCCC_LAUNCH(ev, k_lu_update, dim3(T * T, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lu_rhs(const RhsArgs& a, int n_jobs, hipStream_t st, const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_lu_rhs, dim3((a.N + kRhsB - 1) / kRhsB, n_jobs), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace wpccc

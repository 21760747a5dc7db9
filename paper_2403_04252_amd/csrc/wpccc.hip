// One-centre WP-CCC propagation on gfx950: C ABI, plan and HIP kernels.
//
// Hot path (per RK4 step of Algorithm 1, for every path of the batch):
//   1. slot setup   R = sqrt(b^2+z^2), Theta; Eq. D2 radial integrals at the
//                   exact R for every (a, b, lambda) triple; normalised
//                   associated Legendre functions of cos Theta; the
//                   interaction-picture phases exp(i eps z / v).
//   2. RK4 stages   K_s = M(z_s) u_s with M = -(i/v) Zp D_T (Eq. D1), applied
//                   block-factored (no dense D), fused with the RK4 updates.
//
// Radial integrals at the exact R.  With the grid quadrature of Eq. D2,
//   F(R) = sum_i w_i r_i^2 f_a f_b min(r_i,R)^lam / max(r_i,R)^(lam+1)
//        = R^-(lam+1) A_k + R^lam B_(k+1),
//   A_k = sum_{i<=k} w_i r_i^(2+lam) f_a f_b,  B_k = sum_{i>=k} w_i r_i^(1-lam) f_a f_b,
// where k is the last node with r_k <= R: the kernel min/max^(lam) splits into
// a power of r times a power of R on each side of R.  The partial moments are
// built once per basis (k_moments); per R each integral is two loads and two
// multiplies instead of an n_r-term contraction.  This is the same quadrature
// as the direct sum, in a different association order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "wpccc_impl.h"

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

constexpr int kMaxL = 10;          // largest l of a basis
constexpr int kSlots = 3;          // z, z_mid, z_new

// Per-basis sizes passed to kernels by value.
struct Meta {
    int l_max, lam_max, n_r, n_f, n_states, n_trip, n_pb;
    int n_l[kMaxL + 1];
    int state_off[kMaxL + 1];
};

__host__ __device__ inline int pb_index(int lam, int mu) { return lam * (lam + 1) / 2 + mu; }

// coefficient table index for (l', m', l, m, lambda)
__host__ __device__ inline int coef_index(const Meta& m, int lp, int mp, int l, int mm, int lam) {
    const int L1 = m.l_max + 1, M1 = 2 * m.l_max + 1, Lm = m.lam_max + 1;
    return ((((lp * M1 + (mp + m.l_max)) * L1 + l) * M1 + (mm + m.l_max)) * Lm) + lam;
}

// block table index for (l_a <= l_b, lambda)
__host__ __device__ inline int blk_index(const Meta& m, int la, int lb, int lam) {
    return (la * (m.l_max + 1) + lb) * (m.lam_max + 1) + lam;
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Partial radial moments, one thread per (a, b, lambda) triple.
//   tab[k][t].x = A_k     = sum_{i=1..k}   w_i r_i^(2+lam) f_a(r_i) f_b(r_i)
//   tab[k][t].y = B_(k+1) = sum_{i=k+1..n_r} w_i r_i^(1-lam) f_a(r_i) f_b(r_i)
// phiT is [n_r+1][n_f] so that a wave reads neighbouring functions.
__global__ void k_moments(const double* __restrict__ r, const double* __restrict__ w,
                          const double* __restrict__ phiT, const int* __restrict__ trip_a,
                          const int* __restrict__ trip_b, const int* __restrict__ trip_lam,
                          int n_r, int n_f, int n_trip, double2* __restrict__ tab) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_trip) return;
    const int a = trip_a[t], b = trip_b[t], lam = trip_lam[t];
    double A = 0.0;
    tab[t].x = 0.0;
    for (int i = 1; i <= n_r; ++i) {
        const double ri = r[i];
        double p = ri * ri;
        for (int q = 0; q < lam; ++q) p *= ri;
        A += w[i] * p * phiT[(size_t)i * n_f + a] * phiT[(size_t)i * n_f + b];
        tab[(size_t)i * n_trip + t].x = A;
    }
    double B = 0.0;
    tab[(size_t)n_r * n_trip + t].y = 0.0;
    for (int i = n_r; i >= 1; --i) {
        const double ri = r[i];
        double p = ri;  // r^(1-lam)
        if (lam == 0) {
            p = ri;
        } else {
            double q = 1.0;
            for (int s = 1; s < lam; ++s) q *= ri;
            p = 1.0 / q;
        }
        B += w[i] * p * phiT[(size_t)i * n_f + a] * phiT[(size_t)i * n_f + b];
        tab[(size_t)(i - 1) * n_trip + t].y = B;
    }
}

// Normalised associated Legendre Pbar_l^m = sqrt((l-m)!/(l+m)!) P_l^m (Condon-
// Shortley phase), 0 <= m <= l <= lam_max, written to pb[pb_index(l, m)].
__device__ void legendre_normalised(int lam_max, double x, double* pb) {
    const double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int m = 0; m <= lam_max; ++m) {
        if (m > 0) pmm *= -sqrt((2.0 * m - 1.0) / (2.0 * m)) * s;
        pb[pb_index(m, m)] = pmm;
        if (m + 1 <= lam_max) {
            double p0 = pmm;
            double p1 = sqrt(2.0 * m + 1.0) * x * pmm;
            pb[pb_index(m + 1, m)] = p1;
            for (int l = m + 1; l < lam_max; ++l) {
                const double p2 = ((2.0 * l + 1.0) * x * p1 - sqrt((double)(l + m) * (l - m)) * p0) /
                                  sqrt((double)(l + 1 + m) * (l + 1 - m));
                pb[pb_index(l + 1, m)] = p2;
                p0 = p1;
                p1 = p2;
            }
        }
    }
}

struct SlotJob {
    int n;            // number of slots to fill (1..3)
    int slot[kSlots];
    double z[kSlots];
    int traj0;        // first path of this launch
};

// Per (path, slot): F(R) for every triple, Pbar table, phases exp(i eps z / v).
// grid: x over triple chunks (+ phase chunks), y = slot entry, z = path.
__global__ void k_slot_setup(Meta meta, const double* __restrict__ r, const double2* __restrict__ tab,
                             const int* __restrict__ trip_lam, const double* __restrict__ eps,
                             const double* __restrict__ bvec, const double* __restrict__ vvec,
                             SlotJob job, int n_blk_F, double* __restrict__ F,
                             double* __restrict__ PB, double2* __restrict__ PH,
                             double* __restrict__ Rslot) {
    const int j = job.traj0 + blockIdx.z;
    const int s = job.slot[blockIdx.y];
    const double z = job.z[blockIdx.y];
    const double b = bvec[j], v = vvec[j];
    const double R = sqrt(b * b + z * z);
    const size_t js = (size_t)j * kSlots + s;
    if ((int)blockIdx.x < n_blk_F) {
        // last node with r_k <= R (r_k = r_max (k/n_r)^2)
        __shared__ int ks;
        if (threadIdx.x == 0) {
            const double rmax = r[meta.n_r];
            int k = (int)floor(meta.n_r * sqrt(fmin(R / rmax, 1.0)));
            k = max(0, min(k, meta.n_r));
            while (k < meta.n_r && r[k + 1] <= R) ++k;
            while (k > 0 && r[k] > R) --k;
            ks = k;
        }
        __syncthreads();
        const int k = ks;
        const int t = blockIdx.x * blockDim.x + threadIdx.x;
        if (t < meta.n_trip) {
            const int lam = trip_lam[t];
            double Rl = 1.0;
            for (int q = 0; q < lam; ++q) Rl *= R;
            const double2 ab = tab[(size_t)k * meta.n_trip + t];
            F[js * meta.n_trip + t] = ab.x / (Rl * R) + ab.y * Rl;
        }
        return;
    }
    const int blk = blockIdx.x - n_blk_F;
    if (blk == 0 && threadIdx.x == 0) {
        legendre_normalised(meta.lam_max, z / R, PB + js * meta.n_pb);
        Rslot[js] = R;
    }
    const int i = blk * blockDim.x + threadIdx.x;
    if (i < meta.n_states) {
        double sn, cs;
        sincos(eps[i] * z / v, &sn, &cs);
        PH[js * meta.n_states + i] = make_double2(cs, sn);
    }
}

// Dense couplings H[row][col] = Zp ph_row conj(ph_col) sum_lam c' Pbar F  (Eq. D1).
__global__ void k_couplings_dense(Meta meta, const double* __restrict__ coef,
                                  const int* __restrict__ blk_off, const double* __restrict__ F,
                                  const double* __restrict__ PB, const double2* __restrict__ PH,
                                  double Zp, double2* __restrict__ H) {
    const int N = meta.n_states;
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    if (col >= N) return;
    int lp = 0, l = 0;
    while (lp < meta.l_max && row >= meta.state_off[lp + 1]) ++lp;
    while (l < meta.l_max && col >= meta.state_off[l + 1]) ++l;
    const int rp = row - meta.state_off[lp], rc = col - meta.state_off[l];
    const int mp = rp / meta.n_l[lp] - lp, np = rp % meta.n_l[lp];
    const int m = rc / meta.n_l[l] - l, n = rc % meta.n_l[l];
    const int mu = mp - m, amu = mu < 0 ? -mu : mu;
    double acc = 0.0;
    for (int lam = abs(l - lp); lam <= l + lp; lam += 2) {
        if (amu > lam) continue;
        const double c = coef[coef_index(meta, lp, mp, l, m, lam)];
        if (c == 0.0) continue;
        double f;
        if (lp <= l) f = F[blk_off[blk_index(meta, lp, l, lam)] + np * meta.n_l[l] + n];
        else f = F[blk_off[blk_index(meta, l, lp, lam)] + n * meta.n_l[lp] + np];
        acc += c * PB[pb_index(lam, amu)] * f;
    }
    const double2 w = cmulc(PH[col], PH[row]);  // ph_row * conj(ph_col)
    H[(size_t)row * N + col] = make_double2(Zp * acc * w.x, Zp * acc * w.y);
}

struct StageArgs {
    Meta meta;
    const double* coef;
    const int* blk_off;
    const double* F;      // [n_traj][3][n_trip]
    const double* PB;     // [n_traj][3][n_pb]
    const double2* PH;    // [n_traj][3][N]
    const double* vvec;
    double Zp;
    int n_pad;
    int slot;
    int stage;            // 1..4
    int traj0;
    double h;
    const double2* u_in;  // stage input  [n_traj][n_pad]
    double2* X;           // amplitudes   [n_traj][n_pad]
    double2* Xacc;        // accumulator
    double2* u_out;       // next stage input
    int* flag;            // non-finite latch
};

constexpr int kStageThreads = 256;

// One RK4 stage for one (path, l', m') block of output rows.
//   x' = conj(ph) u;  V^lam_l[n] = sum_m c'(l'm', l m, lam) Pbar_lam^|m'-m| x'_{l m n};
//   y'[n'] = sum_{l, lam, n} F_{(l' n'), (l n), lam} V^lam_l[n];
//   K = -(i/v) Zp ph y'; then the RK4 combination for these rows.
__global__ __launch_bounds__(kStageThreads) void k_stage(StageArgs a) {
    extern __shared__ double2 smem[];
    const Meta& meta = a.meta;
    const int N = meta.n_states;
    const int j = a.traj0 + blockIdx.y;
    const int blk = blockIdx.x;
    int lp = 0;
    while ((lp + 1) * (lp + 1) <= blk) ++lp;
    const int mp = blk - lp * lp - lp;
    const int nlp = meta.n_l[lp];
    const size_t js = (size_t)j * kSlots + a.slot;
    const double* F = a.F + js * meta.n_trip;
    const double* pb = a.PB + js * meta.n_pb;
    const double2* ph = a.PH + js * N;
    const double2* u = a.u_in + (size_t)j * a.n_pad;

    double2* xs = smem;                 // [N]
    double2* V = xs + N;                // [nV]
    // count V entries for this l'
    int nV = 0;
    for (int l = 0; l <= meta.l_max; ++l)
        for (int lam = abs(l - lp); lam <= l + lp; lam += 2) nV += meta.n_l[l];
    int2* vmeta = reinterpret_cast<int2*>(V + nV);  // (F base, F stride over n')

    for (int i = threadIdx.x; i < N; i += blockDim.x) xs[i] = cmulc(ph[i], u[i]);
    __syncthreads();

    for (int e = threadIdx.x; e < nV; e += blockDim.x) {
        int rem = e, l = 0, lam = 0;
        bool found = false;
        for (l = 0; l <= meta.l_max && !found; ++l) {
            for (lam = abs(l - lp); lam <= l + lp; lam += 2) {
                if (rem < meta.n_l[l]) { found = true; break; }
                rem -= meta.n_l[l];
            }
            if (found) break;
        }
        const int n = rem;
        const int nl = meta.n_l[l];
        double2 acc = make_double2(0.0, 0.0);
        const int m_lo = max(-l, mp - lam), m_hi = min(l, mp + lam);
        for (int m = m_lo; m <= m_hi; ++m) {
            const double c = a.coef[coef_index(meta, lp, mp, l, m, lam)];
            if (c == 0.0) continue;
            const int mu = mp - m;
            const double g = c * pb[pb_index(lam, mu < 0 ? -mu : mu)];
            const double2 x = xs[meta.state_off[l] + (m + l) * nl + n];
            acc.x += g * x.x;
            acc.y += g * x.y;
        }
        V[e] = acc;
        int2 mt;
        if (lp <= l) mt = make_int2(a.blk_off[blk_index(meta, lp, l, lam)] + n, nl);
        else mt = make_int2(a.blk_off[blk_index(meta, l, lp, lam)] + n * nlp, 1);
        vmeta[e] = mt;
    }
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n_waves = blockDim.x >> 6;
    const double v = a.vvec[j];
    for (int np = wave; np < nlp; np += n_waves) {
        double re = 0.0, im = 0.0;
        for (int e = lane; e < nV; e += 64) {
            const int2 mt = vmeta[e];
            const double f = F[mt.x + np * mt.y];
            const double2 x = V[e];
            re += f * x.x;
            im += f * x.y;
        }
        for (int off = 32; off > 0; off >>= 1) {
            re += __shfl_down(re, off, 64);
            im += __shfl_down(im, off, 64);
        }
        if (lane == 0) {
            const int row = meta.state_off[lp] + (mp + lp) * nlp + np;
            // K = -(i/v) Zp ph y'
            const double2 py = cmul(ph[row], make_double2(re, im));
            const double sc = a.Zp / v;
            const double2 K = make_double2(sc * py.y, -sc * py.x);
            const size_t o = (size_t)j * a.n_pad + row;
            const double h = a.h;
            const double2 x0 = a.X[o];
            if (a.stage == 1) {
                a.u_out[o] = make_double2(x0.x + 0.5 * h * K.x, x0.y + 0.5 * h * K.y);
                a.Xacc[o] = make_double2(x0.x + h / 6.0 * K.x, x0.y + h / 6.0 * K.y);
            } else if (a.stage == 2 || a.stage == 3) {
                const double c = (a.stage == 2) ? 0.5 * h : h;
                a.u_out[o] = make_double2(x0.x + c * K.x, x0.y + c * K.y);
                const double2 xa = a.Xacc[o];
                a.Xacc[o] = make_double2(xa.x + h / 3.0 * K.x, xa.y + h / 3.0 * K.y);
            } else {
                const double2 xa = a.Xacc[o];
                const double2 xn = make_double2(xa.x + h / 6.0 * K.x, xa.y + h / 6.0 * K.y);
                if (!isfinite(xn.x) || !isfinite(xn.y)) atomicOr(a.flag, 1);
                a.X[o] = xn;
            }
        }
    }
}

// P_i = |X_i|^2 and the norm per path.
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

}  // namespace wpccc

using namespace wpccc;

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------

struct wpccc_plan_s {
    Meta meta{};
    int n_traj = 0, n_pad = 0, batched = 1;
    double Zp = 1.0;
    std::vector<double> b, v;
    int device = 0;
    // device buffers
    double *d_r = nullptr, *d_coef = nullptr, *d_eps = nullptr, *d_b = nullptr, *d_v = nullptr;
    int *d_blk_off = nullptr, *d_trip_lam = nullptr, *d_flag = nullptr;
    double2* d_tab = nullptr;
    double *d_F = nullptr, *d_PB = nullptr, *d_R = nullptr;
    double2 *d_PH = nullptr, *d_Ua = nullptr, *d_Ub = nullptr, *d_Xacc = nullptr;
    long long bytes = 0;
    int stage_smem = 0;
    std::vector<int> blk_off_host;
};

namespace {

template <typename T>
int dev_alloc(T** p, size_t count, long long& total) {
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        set_error("hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
        *p = nullptr;
        return e == hipErrorOutOfMemory ? WPCCC_ENOMEM : WPCCC_EHIP;
    }
    total += (long long)(count * sizeof(T));
    return WPCCC_OK;
}

void free_plan(wpccc_plan_s* p) {
    if (!p) return;
    void* bufs[] = {p->d_r, p->d_coef, p->d_eps, p->d_b, p->d_v, p->d_blk_off, p->d_trip_lam,
                    p->d_flag, p->d_tab, p->d_F, p->d_PB, p->d_R, p->d_PH, p->d_Ua, p->d_Ub,
                    p->d_Xacc};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    delete p;
}

#define TRY(x)                      \
    do {                            \
        int rc_ = (x);              \
        if (rc_ != WPCCC_OK) {      \
            free_plan(plan);        \
            return rc_;             \
        }                           \
    } while (0)

#define HIPTRY(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            set_error("%s failed: %s", #expr, hipGetErrorString(e_));                   \
            free_plan(plan);                                                            \
            return WPCCC_EHIP;                                                          \
        }                                                                               \
    } while (0)

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("launch of %s failed: %s", what, hipGetErrorString(e));
        return WPCCC_EHIP;
    }
    return WPCCC_OK;
}

}  // namespace

extern "C" {

const char* wpccc_last_error(void) { return g_err.c_str(); }

const char* wpccc_version(void) { return "0.1.0"; }

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
        set_error("wpccc_plan_create: the two-centre form is not available in this build");
        return WPCCC_ENOTSUP;
    }
    for (int j = 0; j < n_traj; ++j)
        if (!(b_host[j] > 0.0) || !(v_host[j] > 0.0) || !std::isfinite(b_host[j]) ||
            !std::isfinite(v_host[j])) {
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
    HIPTRY(hipGetDevice(&plan->device));
    plan->n_traj = n_traj;
    plan->batched = o.batched ? 1 : 0;
    plan->Zp = o.Zp;
    plan->b.assign(b_host, b_host + n_traj);
    plan->v.assign(v_host, v_host + n_traj);
    const int N = hb.n_states;
    plan->n_pad = (N + 7) & ~7;

    Meta& m = plan->meta;
    m.l_max = hb.spec.l_max;
    m.lam_max = 2 * m.l_max;
    m.n_r = hb.n_r;
    m.n_f = hb.n_f;
    m.n_states = N;
    m.n_pb = (m.lam_max + 1) * (m.lam_max + 2) / 2;
    for (int l = 0; l <= kMaxL; ++l) {
        m.n_l[l] = l <= m.l_max ? hb.n_l[l] : 0;
        m.state_off[l] = l <= m.l_max ? hb.state_off[l] : N;
    }
    // triple list: blocks (l_a <= l_b, lambda), lambda = |l_a - l_b| .. l_a + l_b step 2
    std::vector<int> ta, tb, tl;
    plan->blk_off_host.assign((size_t)(m.l_max + 1) * (m.l_max + 1) * (m.lam_max + 1), -1);
    for (int la = 0; la <= m.l_max; ++la)
        for (int lb = la; lb <= m.l_max; ++lb)
            for (int lam = lb - la; lam <= la + lb; lam += 2) {
                plan->blk_off_host[blk_index(m, la, lb, lam)] = (int)ta.size();
                for (int ia = 0; ia < hb.n_l[la]; ++ia)
                    for (int ib = 0; ib < hb.n_l[lb]; ++ib) {
                        ta.push_back(hb.rad_off[la] + ia);
                        tb.push_back(hb.rad_off[lb] + ib);
                        tl.push_back(lam);
                    }
            }
    m.n_trip = (int)ta.size();
    // Eq. D1 coefficients c'(l'm', lm, lambda): -sqrt((2l+1)/(2l'+1)) C^{l'0}_{lam0 l0}
    // C^{l'm'}_{lam mu lm}, times (-1)^mu for mu < 0 so that the product with
    // Pbar_lam^|mu| equals the paper's sqrt((lam-mu)!/(lam+mu)!) P_lam^mu.
    const int L1 = m.l_max + 1, M1 = 2 * m.l_max + 1;
    std::vector<double> coef((size_t)L1 * M1 * L1 * M1 * (m.lam_max + 1), 0.0);
    for (int lp = 0; lp <= m.l_max; ++lp)
        for (int mp = -lp; mp <= lp; ++mp)
            for (int l = 0; l <= m.l_max; ++l)
                for (int mm = -l; mm <= l; ++mm)
                    for (int lam = std::abs(l - lp); lam <= l + lp; lam += 2) {
                        const int mu = mp - mm;
                        if (std::abs(mu) > lam) continue;
                        double c = -std::sqrt((2.0 * l + 1.0) / (2.0 * lp + 1.0)) *
                                   clebsch_gordan(lam, 0, l, 0, lp, 0) *
                                   clebsch_gordan(lam, mu, l, mm, lp, mp);
                        if (mu < 0 && (mu % 2)) c = -c;
                        coef[coef_index(m, lp, mp, l, mm, lam)] = c;
                    }
    // phi transposed [n_r+1][n_f]
    std::vector<double> phiT((size_t)(hb.n_r + 1) * hb.n_f);
    for (int a = 0; a < hb.n_f; ++a)
        for (int i = 0; i <= hb.n_r; ++i) phiT[(size_t)i * hb.n_f + a] = hb.phi[(size_t)a * (hb.n_r + 1) + i];

    long long& tot = plan->bytes;
    double *d_w = nullptr, *d_phiT = nullptr;
    int *d_ta = nullptr, *d_tb = nullptr;
    TRY(dev_alloc(&plan->d_r, hb.r.size(), tot));
    TRY(dev_alloc(&plan->d_coef, coef.size(), tot));
    TRY(dev_alloc(&plan->d_eps, (size_t)N, tot));
    TRY(dev_alloc(&plan->d_b, (size_t)n_traj, tot));
    TRY(dev_alloc(&plan->d_v, (size_t)n_traj, tot));
    TRY(dev_alloc(&plan->d_blk_off, plan->blk_off_host.size(), tot));
    TRY(dev_alloc(&plan->d_trip_lam, (size_t)m.n_trip, tot));
    TRY(dev_alloc(&plan->d_flag, 1, tot));
    TRY(dev_alloc(&plan->d_tab, (size_t)(m.n_r + 1) * m.n_trip, tot));
    TRY(dev_alloc(&plan->d_F, (size_t)n_traj * kSlots * m.n_trip, tot));
    TRY(dev_alloc(&plan->d_PB, (size_t)n_traj * kSlots * m.n_pb, tot));
    TRY(dev_alloc(&plan->d_R, (size_t)n_traj * kSlots, tot));
    TRY(dev_alloc(&plan->d_PH, (size_t)n_traj * kSlots * N, tot));
    TRY(dev_alloc(&plan->d_Ua, (size_t)n_traj * plan->n_pad, tot));
    TRY(dev_alloc(&plan->d_Ub, (size_t)n_traj * plan->n_pad, tot));
    TRY(dev_alloc(&plan->d_Xacc, (size_t)n_traj * plan->n_pad, tot));
    long long tmp_bytes = 0;
    auto free_tmp = [&]() {
        if (d_w) (void)hipFree(d_w);
        if (d_phiT) (void)hipFree(d_phiT);
        if (d_ta) (void)hipFree(d_ta);
        if (d_tb) (void)hipFree(d_tb);
    };
    int rc = dev_alloc(&d_w, hb.w.size(), tmp_bytes);
    if (rc == WPCCC_OK) rc = dev_alloc(&d_phiT, phiT.size(), tmp_bytes);
    if (rc == WPCCC_OK) rc = dev_alloc(&d_ta, ta.size(), tmp_bytes);
    if (rc == WPCCC_OK) rc = dev_alloc(&d_tb, tb.size(), tmp_bytes);
    if (rc != WPCCC_OK) {
        free_tmp();
        free_plan(plan);
        return rc;
    }
    hipError_t e = hipSuccess;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    up(plan->d_r, hb.r.data(), hb.r.size() * sizeof(double));
    up(d_w, hb.w.data(), hb.w.size() * sizeof(double));
    up(d_phiT, phiT.data(), phiT.size() * sizeof(double));
    up(plan->d_coef, coef.data(), coef.size() * sizeof(double));
    up(plan->d_eps, hb.eps.data(), (size_t)N * sizeof(double));
    up(plan->d_b, b_host, (size_t)n_traj * sizeof(double));
    up(plan->d_v, v_host, (size_t)n_traj * sizeof(double));
    up(plan->d_blk_off, plan->blk_off_host.data(), plan->blk_off_host.size() * sizeof(int));
    up(plan->d_trip_lam, tl.data(), tl.size() * sizeof(int));
    up(d_ta, ta.data(), ta.size() * sizeof(int));
    up(d_tb, tb.data(), tb.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(plan->d_flag, 0, sizeof(int), st);
    if (e == hipSuccess) {
        const int nb = (m.n_trip + 127) / 128;
        hipLaunchKernelGGL(k_moments, dim3(nb), dim3(128), 0, st, plan->d_r, d_w, d_phiT, d_ta, d_tb,
                           plan->d_trip_lam, m.n_r, m.n_f, m.n_trip, plan->d_tab);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    free_tmp();
    if (e != hipSuccess) {
        set_error("wpccc_plan_create: device setup failed: %s", hipGetErrorString(e));
        free_plan(plan);
        return WPCCC_EHIP;
    }
    // stage kernel LDS: x' [N] + V [nV] (complex) + V meta [nV] (int2)
    int nv_max = 0;
    for (int lp = 0; lp <= m.l_max; ++lp) {
        int nV = 0;
        for (int l = 0; l <= m.l_max; ++l)
            for (int lam = std::abs(l - lp); lam <= l + lp; lam += 2) nV += m.n_l[l];
        nv_max = std::max(nv_max, nV);
    }
    plan->stage_smem = (int)(N * sizeof(double2) + nv_max * (sizeof(double2) + sizeof(int2)));
    if (plan->stage_smem > 160 * 1024) {
        set_error("wpccc_plan_create: basis too large for the stage kernel's LDS (%d bytes)",
                  plan->stage_smem);
        free_plan(plan);
        return WPCCC_EINVAL;
    }
    if (plan->stage_smem > 64 * 1024) {
        hipError_t ea = hipFuncSetAttribute((const void*)k_stage,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            plan->stage_smem);
        if (ea != hipSuccess) {
            set_error("hipFuncSetAttribute failed: %s", hipGetErrorString(ea));
            free_plan(plan);
            return WPCCC_EHIP;
        }
    }
    *out = plan;
    return WPCCC_OK;
}

int wpccc_plan_info(wpccc_plan_t plan, int* n_traj, int* n_states, int* n_pad, long long* device_bytes) {
    if (!plan) {
        set_error("wpccc_plan_info: NULL plan");
        return WPCCC_EINVAL;
    }
    if (n_traj) *n_traj = plan->n_traj;
    if (n_states) *n_states = plan->meta.n_states;
    if (n_pad) *n_pad = plan->n_pad;
    if (device_bytes) *device_bytes = plan->bytes;
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
    int flag = 0;
    WPCCC_HIP_CHECK(hipMemcpyAsync(&flag, plan->d_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    WPCCC_HIP_CHECK(hipStreamSynchronize(st));
    WPCCC_HIP_CHECK(hipMemsetAsync(plan->d_flag, 0, sizeof(int), st));
    if (flag) {
        set_error("non-finite amplitude detected during propagation");
        return WPCCC_ENUMERIC;
    }
    return WPCCC_OK;
}

}  // extern "C"

namespace {

// Enqueue the slot setup for paths [j0, j0 + nj).
int launch_setup(wpccc_plan_s* p, const SlotJob& job, int nj, hipStream_t st) {
    const Meta& m = p->meta;
    const int nbF = (m.n_trip + 255) / 256;
    const int nbP = (m.n_states + 255) / 256;
    hipLaunchKernelGGL(k_slot_setup, dim3(nbF + nbP, job.n, nj), dim3(256), 0, st, m, p->d_r, p->d_tab,
                       p->d_trip_lam, p->d_eps, p->d_b, p->d_v, job, nbF, p->d_F, p->d_PB, p->d_PH, p->d_R);
    return check_launch("k_slot_setup");
}

int launch_stage(wpccc_plan_s* p, int j0, int nj, int stage, int slot, double h, const double2* u_in,
                 double2* X, double2* u_out, hipStream_t st) {
    StageArgs a;
    a.meta = p->meta;
    a.coef = p->d_coef;
    a.blk_off = p->d_blk_off;
    a.F = p->d_F;
    a.PB = p->d_PB;
    a.PH = p->d_PH;
    a.vvec = p->d_v;
    a.Zp = p->Zp;
    a.n_pad = p->n_pad;
    a.slot = slot;
    a.stage = stage;
    a.traj0 = j0;
    a.h = h;
    a.u_in = u_in;
    a.X = X;
    a.Xacc = p->d_Xacc;
    a.u_out = u_out;
    a.flag = p->d_flag;
    const int nblk = (p->meta.l_max + 1) * (p->meta.l_max + 1);
    hipLaunchKernelGGL(k_stage, dim3(nblk, nj), dim3(kStageThreads), p->stage_smem, st, a);
    return check_launch("k_stage");
}

// One RK4 step z -> z + h for paths [j0, j0+nj); slots: sz (z), sm (mid), sn (new).
int enqueue_step(wpccc_plan_s* p, double2* X, int j0, int nj, double h, int sz, int sm, int sn,
                 hipStream_t st) {
    int rc;
    if ((rc = launch_stage(p, j0, nj, 1, sz, h, X, X, p->d_Ua, st))) return rc;
    if ((rc = launch_stage(p, j0, nj, 2, sm, h, p->d_Ua, X, p->d_Ub, st))) return rc;
    if ((rc = launch_stage(p, j0, nj, 3, sm, h, p->d_Ub, X, p->d_Ua, st))) return rc;
    if ((rc = launch_stage(p, j0, nj, 4, sn, h, p->d_Ua, X, nullptr, st))) return rc;
    return WPCCC_OK;
}

bool path_hits_origin(const wpccc_plan_s* p, double z) {
    for (double b : p->b)
        if (!(std::sqrt(b * b + z * z) > 0.0)) return true;
    return false;
}

}  // namespace

extern "C" {

int wpccc_couplings(wpccc_plan_t plan, int j, double z, void* H_dev, void* S_dev, void* stream) {
    clear_error();
    if (!plan || !H_dev || j < 0 || j >= plan->n_traj || !std::isfinite(z)) {
        set_error("wpccc_couplings: bad plan, path index or z");
        return WPCCC_EINVAL;
    }
    if (S_dev) {
        set_error("wpccc_couplings: S_dev must be NULL for a one-centre plan");
        return WPCCC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    SlotJob job{};
    job.n = 1;
    job.slot[0] = 0;
    job.z[0] = z;
    job.traj0 = j;
    int rc = launch_setup(plan, job, 1, st);
    if (rc) return rc;
    const Meta& m = plan->meta;
    const size_t js = (size_t)j * kSlots;
    hipLaunchKernelGGL(k_couplings_dense, dim3((m.n_states + 127) / 128, m.n_states), dim3(128), 0, st, m,
                       plan->d_coef, plan->d_blk_off, plan->d_F + js * m.n_trip, plan->d_PB + js * m.n_pb,
                       plan->d_PH + js * m.n_states, plan->Zp, (double2*)H_dev);
    return check_launch("k_couplings_dense");
}

int wpccc_step(wpccc_plan_t plan, void* X_dev, double z, double h, void* stream) {
    clear_error();
    if (!plan || !X_dev || !(h != 0.0) || !std::isfinite(z) || !std::isfinite(h)) {
        set_error("wpccc_step: bad plan, X_dev, z or h");
        return WPCCC_EINVAL;
    }
    if (path_hits_origin(plan, z) || path_hits_origin(plan, z + 0.5 * h) || path_hits_origin(plan, z + h)) {
        set_error("wpccc_step: R = 0 on the step");
        return WPCCC_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    double2* X = (double2*)X_dev;
    const int chunk = plan->batched ? plan->n_traj : 1;
    for (int j0 = 0; j0 < plan->n_traj; j0 += chunk) {
        const int nj = std::min(chunk, plan->n_traj - j0);
        SlotJob job{};
        job.n = 3;
        job.traj0 = j0;
        job.slot[0] = 0; job.z[0] = z;
        job.slot[1] = 1; job.z[1] = z + 0.5 * h;
        job.slot[2] = 2; job.z[2] = z + h;
        int rc = launch_setup(plan, job, nj, st);
        if (rc) return rc;
        if ((rc = enqueue_step(plan, X, j0, nj, h, 0, 1, 2, st))) return rc;
    }
    return WPCCC_OK;
}

int wpccc_propagate(wpccc_plan_t plan, const double* zgrid_host, int n_points, void* X_dev, void* P_dev,
                    void* norm_dev, void* stream) {
    clear_error();
    if (!plan || !zgrid_host || !X_dev || n_points < 2) {
        set_error("wpccc_propagate: bad plan, grid or X_dev (need >= 2 points)");
        return WPCCC_EINVAL;
    }
    for (int i = 0; i < n_points; ++i) {
        if (!std::isfinite(zgrid_host[i]) || (i > 0 && !(zgrid_host[i] > zgrid_host[i - 1]))) {
            set_error("wpccc_propagate: z-grid must be finite and strictly increasing");
            return WPCCC_EINVAL;
        }
    }
    for (int i = 0; i < n_points; ++i) {
        if (path_hits_origin(plan, zgrid_host[i]) ||
            (i + 1 < n_points && path_hits_origin(plan, 0.5 * (zgrid_host[i] + zgrid_host[i + 1])))) {
            set_error("wpccc_propagate: R = 0 on the grid");
            return WPCCC_EINVAL;
        }
    }
    hipStream_t st = (hipStream_t)stream;
    double2* X = (double2*)X_dev;
    const int chunk = plan->batched ? plan->n_traj : 1;
    for (int j0 = 0; j0 < plan->n_traj; j0 += chunk) {
        const int nj = std::min(chunk, plan->n_traj - j0);
        // M at the first grid point
        SlotJob first{};
        first.n = 1;
        first.traj0 = j0;
        first.slot[0] = 0;
        first.z[0] = zgrid_host[0];
        int rc = launch_setup(plan, first, nj, st);
        if (rc) return rc;
        int sz = 0, sn = 2;
        for (int i = 0; i + 1 < n_points; ++i) {
            const double z = zgrid_host[i], zn = zgrid_host[i + 1];
            const double h = zn - z;
            SlotJob job{};
            job.n = 2;
            job.traj0 = j0;
            job.slot[0] = 1; job.z[0] = 0.5 * (z + zn);
            job.slot[1] = sn; job.z[1] = zn;
            if ((rc = launch_setup(plan, job, nj, st))) return rc;
            if ((rc = enqueue_step(plan, X, j0, nj, h, sz, 1, sn, st))) return rc;
            std::swap(sz, sn);  // M(z_new) becomes M(z) of the next step
        }
    }
    if (P_dev || norm_dev) {
        hipLaunchKernelGGL(k_probabilities, dim3(plan->n_traj), dim3(256), 0, st, (const double2*)X,
                           plan->meta.n_states, plan->n_pad, (double*)P_dev, (double*)norm_dev);
        int rc = check_launch("k_probabilities");
        if (rc) return rc;
    }
    return WPCCC_OK;
}

}  // extern "C"

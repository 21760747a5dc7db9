// Observables at the end of a propagation (Sec. II after Algorithm 1 and
// Sec. III): the probabilities of the reaction channels per path and the
// cross sections of a batch of impact parameters.
//
// Channels: the state each amplitude belongs to decides its channel, from the
// centre it is expanded about and the sign of its energy (bound eigenstates
// below zero, wave-packet pseudostates above):
//   elastic (target state 0), target excitation (other target states with
//   eps < 0), target continuum (eps > 0), capture (projectile states with
//   eps < 0, two-centre only), projectile continuum (eps > 0), and the total.
// The codes are set once per plan on the host; k_channels sums P per code.
// Cross section of a channel over the paths of one group (paths sharing the
// basis pair and the speed): sigma = 2 pi int_0^inf P(b) b db by the
// trapezoidal rule over the group's impact parameters in increasing order,
// with the integrand 0 at b = 0 and nothing beyond the largest b.
#include <hip/hip_runtime.h>

#include "plan.h"

namespace wpccc {

namespace {

constexpr int kObsThreads = 256;

// One workgroup per path: chan[j][c] = sum of P[j][i] over the states i with
// code c (c < kNumChannels - 1), chan[j][kNumChannels - 1] = sum over every
// state.  Each thread sums a strided part in index order, the partial sums
// are added by a fixed tree: the result does not depend on scheduling.
__global__ __launch_bounds__(kObsThreads) void k_channels(const double* __restrict__ P,
                                                          const unsigned char* __restrict__ code, int n_pad,
                                                          double* __restrict__ chan) {
    __shared__ double red[kNumChannels][kObsThreads];
    const int j = blockIdx.x, t = threadIdx.x;
    double acc[kNumChannels];
#pragma unroll
    for (int c = 0; c < kNumChannels; ++c) acc[c] = 0.0;
    const double* p = P + (size_t)j * n_pad;
    const unsigned char* cd = code + (size_t)j * n_pad;
    for (int i = t; i < n_pad; i += kObsThreads) {
        const int c = cd[i];
        if (c >= kNumChannels - 1) continue;   // padding entry
        const double v = p[i];
#pragma unroll
        for (int k = 0; k < kNumChannels - 1; ++k)
            if (c == k) acc[k] += v;
        acc[kNumChannels - 1] += v;
    }
#pragma unroll
    for (int c = 0; c < kNumChannels; ++c) red[c][t] = acc[c];
    __syncthreads();
    for (int w = kObsThreads / 2; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int c = 0; c < kNumChannels; ++c) red[c][t] += red[c][t + w];
        __syncthreads();
    }
    if (t < kNumChannels) chan[(size_t)j * kNumChannels + t] = red[t][0];
}

// One thread per (group g, channel c): the trapezoidal rule over the group's
// paths order[gstart[g] .. gstart[g+1]) (sorted by b), from b = 0.
__global__ void k_cross_sections(const double* __restrict__ chan, const double* __restrict__ b,
                                 const int* __restrict__ order, const int* __restrict__ gstart, int n_groups,
                                 double* __restrict__ sigma) {
    const int g = blockIdx.x, c = threadIdx.x;
    if (g >= n_groups || c >= kNumChannels) return;
    double b0 = 0.0, f0 = 0.0, total = 0.0;
    for (int k = gstart[g]; k < gstart[g + 1]; ++k) {
        const int j = order[k];
        const double b1 = b[j];
        const double f1 = chan[(size_t)j * kNumChannels + c] * b1;
        total += 0.5 * (b1 - b0) * (f0 + f1);
        b0 = b1;
        f0 = f1;
    }
    sigma[(size_t)g * kNumChannels + c] = 2.0 * M_PI * total;
}

}  // namespace

int obs_build(Observables& o, int n_traj, int n_pad, const std::vector<unsigned char>& codes,
              const std::vector<int>& group_of, const std::vector<double>& b) {
    o.n_traj = n_traj;
    o.n_pad = n_pad;
    o.group_of = group_of;
    o.n_groups = 0;
    for (int g : group_of) o.n_groups = std::max(o.n_groups, g + 1);
    // paths of each group by increasing b (stable: equal b keep their order)
    std::vector<int> order;
    std::vector<int> gstart(1, 0);
    for (int g = 0; g < o.n_groups; ++g) {
        std::vector<int> mine;
        for (int j = 0; j < n_traj; ++j)
            if (group_of[j] == g) mine.push_back(j);
        std::stable_sort(mine.begin(), mine.end(), [&](int x, int y) { return b[x] < b[y]; });
        order.insert(order.end(), mine.begin(), mine.end());
        gstart.push_back((int)order.size());
    }
    long long tot = 0;
    int rc = WPCCC_OK;
    auto A = [&](int r) {
        if (rc == WPCCC_OK) rc = r;
    };
    A(dev_alloc(&o.d_code, codes.size(), tot));
    A(dev_alloc(&o.d_order, order.size(), tot));
    A(dev_alloc(&o.d_gstart, gstart.size(), tot));
    A(dev_alloc(&o.d_b, b.size(), tot));
    if (rc) {
        obs_free(o);
        return rc;
    }
    hipError_t e = hipMemcpy(o.d_code, codes.data(), codes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(o.d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(o.d_gstart, gstart.data(), gstart.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(o.d_b, b.data(), b.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        set_error("observable tables: %s", hipGetErrorString(e));
        obs_free(o);
        return WPCCC_EHIP;
    }
    o.bytes = tot;
    return WPCCC_OK;
}

void obs_free(Observables& o) {
    void* bufs[] = {o.d_code, o.d_order, o.d_gstart, o.d_b};
    for (void* q : bufs)
        if (q) (void)hipFree(q);
    o = Observables{};
}

hipError_t launch_observables(const Observables& o, const double* P, double* chan, double* sigma, hipStream_t st,
                              const LaunchEv& ev) {
    WPCCC_LAUNCH(ev, k_channels, dim3(o.n_traj), dim3(kObsThreads), 0, st, P, o.d_code, o.n_pad, chan);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !sigma) return e;
    hipLaunchKernelGGL(k_cross_sections, dim3(o.n_groups), dim3(64), 0, st, chan, o.d_b, o.d_order, o.d_gstart,
                       o.n_groups, sigma);
    return hipGetLastError();
}

}  // namespace wpccc

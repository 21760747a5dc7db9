// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/wpccc.h"

namespace wpccc {

void set_error(const char* fmt, ...);
void clear_error();

// Host-side basis: grid, orthonormal radial functions and the state list.
struct HostBasis {
    wpccc_basis_spec spec{};
    int n_r = 0;                       // grid intervals; n_r + 1 nodes
    std::vector<double> r, w;          // [n_r + 1]
    int n_f = 0;                       // radial functions
    std::vector<double> phi;           // [n_f][n_r + 1]
    std::vector<int> rad_l;            // [n_f]
    std::vector<double> rad_eps;       // [n_f]
    std::vector<int> n_l, rad_off;     // per l
    int n_states = 0;
    std::vector<int> st_l, st_m, st_i; // per state: l, m, radial index
    std::vector<double> eps;           // per state
    std::vector<int> state_off;        // per l: first state of the l block
};

int build_host_basis(const wpccc_basis_spec& spec, HostBasis& out);

// Clebsch-Gordan coefficient <j1 m1 j2 m2 | J M> (Racah's closed formula).
double clebsch_gordan(int j1, int m1, int j2, int m2, int J, int M);

}  // namespace wpccc

struct wpccc_basis_s {
    wpccc::HostBasis hb;
};

#define WPCCC_HIP_CHECK(expr)                                                   \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) {                                                 \
            wpccc::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                               \
            return WPCCC_EHIP;                                                  \
        }                                                                       \
    } while (0)

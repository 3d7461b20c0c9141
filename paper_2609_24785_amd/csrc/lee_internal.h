// Internal declarations shared by the host builder (plain C++) and the device
// side (HIP).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/lee.h"

namespace lee {

constexpr int FRAME = 5;        // zero frame rows above/below the domain
constexpr int LPAD = 8;         // zero columns left of column 0 (alignment)
constexpr int RPAD_MIN = 264;   // columns right of the domain covering strip overrun

struct Host {
    // description
    lee_case_desc d{};
    double dt = 0.0;
    int reach = 5;
    // mask and rows
    std::vector<uint8_t> fluid;        // ny * nx
    std::vector<int32_t> iv;           // ny * 4: [a0, b0, a1, b1) fluid column intervals
    int64_t fluid_nodes = 0;
    // ghosts
    bool built = false;
    std::vector<int32_t> gidx;         // linear j * nx + i, ascending
    std::vector<double> bx, by, gnx, gny, r;
    std::vector<int32_t> cptr, cidx;   // CSR, linear indices
    std::vector<int8_t> deg;
    std::vector<uint8_t> cut;
    std::vector<double> w4;            // 4 per entry: BP, free, Dirichlet, Neumann
    std::vector<double> beta;          // 2 per ghost: beta_D, beta_N
    // ADE (Sec. 2.5): kind 0 rigid, 1 complex pair, 2 real poles
    int ade_kind = 0;
    double ade[4] = {0, 0, 0, 0};      // complex: a, b, 2B1, -2C1 ; real: l1, l2, A1, A2
    // kind 3 (multi-pole, Sec. 2.3): ns states, state k advanced as
    // dX_k = a_k X_k + bn_k X_{k+1} + bp_k X_{k-1} + f_k p_BP, u_n = sum c_k X_k
    int ade_ns = 2;
    double ade_st[8][5] = {};          // per state: a, bn, bp, f, c
    double poles[4] = {0, 0, 0, 0};
    // recorded probes
    int np = 0;
    std::vector<int32_t> probe_ij;     // 2 per probe (origin i0, j0)
    std::vector<double> probe_w;       // 16 per probe, [b * 4 + a]
    int64_t trace_cap = 0;
    double dft_omega = 0.0;
    int64_t dft_start = 0, dft_count = 0;
    // watched ghost: p_BP, u_n,BP and the fluid's u_n at the boundary point,
    // of every step's first stage
    int watch_g = -1;
    int64_t watch_cap = 0;
};

void set_error(const std::string &msg);
lee_status fail(lee_status s, const std::string &msg);

lee_status host_setup(const lee_case_desc *d, Host *h);
lee_status host_build(Host *h, const lee_impedance *z, int degree, lee_ghost_summary *out);
lee_status host_probe_stencil(const Host *h, double x, double y, int32_t *i0, int32_t *j0,
                              double w[16]);

}  // namespace lee

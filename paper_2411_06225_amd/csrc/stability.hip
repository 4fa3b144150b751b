// stability.hip -- the stability pre-check of the propagators F and G.
//
// Sec. 6 warns that an unsuitable coarse solver stalls the iteration; an
// explicit Runge-Kutta step is only meaningful while dt times the spectral
// radius of the Jacobian of h stays inside the method's stability region.
// The check bounds that spectral radius from the grid, the physical
// parameters and the initial state, split into a real part rho_r (diffusion,
// reaction, the dissipative Rusanov operator) and an imaginary part rho_i
// (central-difference advection), and returns dt / dt_max:
//   forward Euler : dt_max = 2 / rho_r, and where rho_i > 0 also
//                   rho_r / (2 rho_i^2) (the classical forward-time
//                   centred-space condition dt <= 2 nu / u^2);
//   classical RK4 : dt_max = 2.78 / (rho_r + rho_i) (the region reaches
//                   -2.785 on the real axis and +-2.83 i on the imaginary);
//   eighth-order  : dt_max = 2.9 / (rho_r + rho_i) (Cooper and Verner's
//                   method: -3.71 and +-3.00 i).
// Bounds per right-hand side, u_max = ||u0||_inf:
//   Burgers        rho_r = 4 nu / dx^2, rho_i = u_max / dx;
//   diffusion-reaction  rho_r = max(Du, Dv) (4/dx^2 + 4/dy^2) + 2 + 3 u_max^2
//                  (the reaction Jacobian's infinity norm);
//   Brusselator    rho_r = max(Du, Dv) (4/dx^2 + 4/dy^2 (+ 4/dz^2 in 3D))
//                  + B + 1 + 3 u_max^2;
//   shallow water  rho_r = 2 a (1/dx + 1/dy), a the largest wave speed
//                  |velocity| + sqrt(g h) of the initial state.
// All bounds are estimates at t0 (the nonlinear systems change their
// Jacobian as they evolve).
#include "plan.h"

namespace rpr {

void stability_bounds(const Geom &g, double umax, double speed, double *rho_r, double *rho_i)
{
    const double lap = 4.0 * g.idx2 + (g.kind == RPR_BURGERS1D ? 0.0 : 4.0 * g.idy2) + 4.0 * g.idz2;
    double rr = 0.0, ri = 0.0;
    switch (g.kind) {
    case RPR_BURGERS1D:
        rr = 4.0 * g.p[0] * g.idx2;
        ri = umax * g.idx;
        break;
    case RPR_DIFFREACT2D:
        rr = std::max(g.p[0], g.p[1]) * lap + 2.0 + 3.0 * umax * umax;
        break;
    case RPR_BRUSS2D:
    case RPR_BRUSS3D:
        rr = std::max(g.p[2], g.p[3]) * lap + g.p[1] + 1.0 + 3.0 * umax * umax;
        break;
    case RPR_SWE2D:
        rr = 2.0 * speed * (g.idx + g.idy);
        break;
    default: break;
    }
    *rho_r = rr;
    *rho_i = ri;
}

double stability_ratio(const Geom &g, int method, double dt, double umax, double speed)
{
    double rr, ri;
    stability_bounds(g, umax, speed, &rr, &ri);
    dt = std::fabs(dt);
    if (method == RPR_RK4 || method == RPR_RK8) {
        // RK4 reaches -2.785 and +-2.83 i, the eighth-order method -3.71 and
        // +-3.00 i (its stability function)
        const double r = rr + ri;
        return r > 0.0 ? dt * r / (method == RPR_RK4 ? 2.78 : 2.9) : 0.0;
    }
    double ratio = rr > 0.0 ? dt * rr / 2.0 : 0.0;
    if (ri > 0.0) {
        // forward Euler amplifies pure advection at any step
        if (!(rr > 0.0)) return INFINITY;
        ratio = std::max(ratio, dt * 2.0 * ri * ri / rr);
    }
    return ratio;
}

}  // namespace rpr

extern "C" rpr_status rpr_stability(const rpr_rhs *h, int32_t d, const rpr_propagator *P, double dt, double umax,
                                    double speed, double *ratio)
{
    Geom g;
    RPR_TRY(make_geom(h, d, &g));
    RPR_TRY(check_prop(P, "P"));
    if (!ratio) return fail(RPR_ERR_INVALID_ARG, "ratio is NULL");
    if (!is_finite(dt) || !(umax >= 0) || !is_finite(umax) || !(speed >= 0) || !is_finite(speed))
        return fail(RPR_ERR_INVALID_ARG, "dt, umax and speed must be finite, umax and speed >= 0");
    *ratio = stability_ratio(g, P->method, dt, umax, speed);
    return RPR_OK;
}

// Conservative caller-side forces summed per body: the soft marker-wall
// repulsion of eq. Usoft (Sec. V.A; App. A applies it between every blob and
// both walls of the slit) and a constant force on every marker (the buoyant
// weight of App. A).
#include "common.h"

namespace rb {

// -dPhi/dr of eq. Usoft: Phi0/b inside r < d, (Phi0/b) exp((d - r)/b) beyond
__device__ __forceinline__ double soft_push(double r, double phi0, double d, double b) {
    return r < d ? phi0 / b : (phi0 / b) * exp((d - r) / b);
}

// FT[p] = [sum_i f_i ; sum_i d_i x f_i], f_i the force on marker i of body p,
// d_i = R(theta_p) r_i^ref.  One thread per body (bodies hold few markers).
__global__ void k_body_forces(const RepDev *reps, const int *body_rep, const int *body_off, int nb,
                              const double *q, const double *theta, const double *rref, double phi0, double d,
                              double b, double fx, double fy, double fz, double *FT) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    const RepDev &R = reps[body_rep[p]];
    double Rm[9];
    quat_to_R(theta + 4 * p, Rm);
    double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
    for (int m = body_off[p]; m < body_off[p + 1]; ++m) {
        const double *rr = rref + 3 * m;
        double dd[3], f[3] = {fx, fy, fz};
        for (int a = 0; a < 3; ++a) {
            dd[a] = (Rm[3 * a] * rr[0] + Rm[3 * a + 1] * rr[1]) + Rm[3 * a + 2] * rr[2];
            if (R.bc[a] == RBFIB_PERIODIC) continue;
            const double x = q[3 * p + a] + dd[a], L = (double)R.n[a] * R.h;
            f[a] += soft_push(x, phi0, d, b) - soft_push(L - x, phi0, d, b);
        }
        for (int a = 0; a < 3; ++a) F[a] += f[a];
        T[0] += dd[1] * f[2] - dd[2] * f[1];
        T[1] += dd[2] * f[0] - dd[0] * f[2];
        T[2] += dd[0] * f[1] - dd[1] * f[0];
    }
    for (int a = 0; a < 3; ++a) {
        FT[6 * p + a] = F[a];
        FT[6 * p + 3 + a] = T[a];
    }
}

void launch_body_forces(Ctx &c, const double *q, const double *theta, double phi0, double d, double b,
                        const double fconst[3], double *FT) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_body_forces, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_reps, c.d_body_rep,
                       c.d_body_off, c.nb, q, theta, c.d_rref, phi0, d, b, fconst[0], fconst[1], fconst[2], FT);
}

}  // namespace rb

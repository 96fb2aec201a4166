// Gradient of a loss L(U) through the mobility solve (differentiating eqs. D1-D4).
//
// With x = (v, pi, lambda, U) the forward solution and (v-bar, pi-bar, lambda', U')
// the solution of the same system with right side (0, 0, 0, dV * U-bar) (the
// operator equals P A P^-1 transposed, P = diag(1, 1, 1/dV, 1/dV)), put
// lambda-bar = lambda'/dV and U-hat = U'/dV.  Then dL/dF = U-hat and, per marker i
// of body p,
//   G_i = grad_r [ lambda-bar_i . (J v)_i ] + (1/dV) grad_r [ lambda_i . (J v-bar)_i ]
//   E_i = -(lambda-bar_i x omega_p) - (lambda_i x omega-hat_p)
//   dL/dq_p = sum_i G_i,   dL/dphi_p = sum_i d_i x (G_i + E_i)
// (phi a lab-frame rotation vector; K depends only on d_i = R(theta_p) r_i^ref).
// For unit quaternions, dL/dtheta = M(theta)^T dL/dphi with
// dphi = 2 vec(dtheta (x) conj(theta)).
#include "common.h"

namespace rb {

template <int W>
__global__ void k_body_grad(const RepDev *reps, const int *body_rep, const int *body_off, const double *r,
                            const double *d, const double *__restrict__ x, const double *__restrict__ xa,
                            const double *theta, double *dFT, double *dq, double *dphi, double *dtheta) {
    extern __shared__ double sred[];   // [nmp][6]
    int p = blockIdx.x;
    const RepDev &R = reps[body_rep[p]];
    int m0 = body_off[p], nmp = body_off[p + 1] - m0;
    double inv_dV = 1.0 / R.dV;
    long long lam0 = R.off + 4 * R.N;
    long long U0 = lam0 + 3LL * R.nm + 6LL * (p - R.b0);
    double om[3] = {x[U0 + 3], x[U0 + 4], x[U0 + 5]};
    double omh[3] = {xa[U0 + 3] * inv_dV, xa[U0 + 4] * inv_dV, xa[U0 + 5] * inv_dV};
    for (int i = threadIdx.x; i < nmp; i += blockDim.x) {
        int m = m0 + i;
        const double *rm = r + 3 * m, *dm = d + 3 * m;
        long long ls = lam0 + 3LL * (m - R.m0);
        double lam[3] = {x[ls], x[ls + 1], x[ls + 2]};
        double lb[3] = {xa[ls] * inv_dV, xa[ls + 1] * inv_dV, xa[ls + 2] * inv_dV};
        double G[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 3; ++c) {
            double g1[3], g2[3];
            interp_grad<W>(R, rm, c, x + R.off + c * R.N, g1);
            interp_grad<W>(R, rm, c, xa + R.off + c * R.N, g2);
            for (int a = 0; a < 3; ++a) G[a] += lb[c] * g1[a] + inv_dV * lam[c] * g2[a];
        }
        double E[3] = {-(lb[1] * om[2] - lb[2] * om[1]) - (lam[1] * omh[2] - lam[2] * omh[1]),
                       -(lb[2] * om[0] - lb[0] * om[2]) - (lam[2] * omh[0] - lam[0] * omh[2]),
                       -(lb[0] * om[1] - lb[1] * om[0]) - (lam[0] * omh[1] - lam[1] * omh[0])};
        double T[3] = {G[0] + E[0], G[1] + E[1], G[2] + E[2]};
        sred[6 * i + 0] = G[0];
        sred[6 * i + 1] = G[1];
        sred[6 * i + 2] = G[2];
        sred[6 * i + 3] = dm[1] * T[2] - dm[2] * T[1];
        sred[6 * i + 4] = dm[2] * T[0] - dm[0] * T[2];
        sred[6 * i + 5] = dm[0] * T[1] - dm[1] * T[0];
    }
    __syncthreads();
    __shared__ double tot[6];
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int i = 0; i < nmp; ++i) s += sred[6 * i + threadIdx.x];
        tot[threadIdx.x] = s;
        if (dFT) dFT[6 * p + threadIdx.x] = xa[U0 + threadIdx.x] * inv_dV;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (dq) for (int a = 0; a < 3; ++a) dq[3 * p + a] = tot[a];
        if (dphi) for (int a = 0; a < 3; ++a) dphi[3 * p + a] = tot[3 + a];
        if (dtheta) {
            const double *th = theta + 4 * p;
            const double *g = tot + 3;
            dtheta[4 * p + 0] = -2.0 * (th[1] * g[0] + th[2] * g[1] + th[3] * g[2]);
            double cx = th[2] * g[2] - th[3] * g[1], cy = th[3] * g[0] - th[1] * g[2], cz = th[1] * g[1] - th[2] * g[0];
            dtheta[4 * p + 1] = 2.0 * (th[0] * g[0] - cx);
            dtheta[4 * p + 2] = 2.0 * (th[0] * g[1] - cy);
            dtheta[4 * p + 3] = 2.0 * (th[0] * g[2] - cz);
        }
    }
}

void launch_body_grad(Ctx &c, const double *x, const double *xa, const double *theta, double *dFT, double *dq,
                      double *dphi, double *dtheta) {
    if (c.nb == 0) return;
    size_t sh = sizeof(double) * 6 * (size_t)c.max_body_nm;
    hipLaunchKernelGGL(c.kw == 6 ? k_body_grad<6> : k_body_grad<4>, dim3(c.nb), dim3(64), sh, c.stream, c.d_reps,
                       c.d_body_rep, c.d_body_off, c.ms[0].r, c.ms[0].d, x, xa, theta, dFT, dq, dphi, dtheta);
}

// b_U[p] = dV * Ubar[p] (right side of the adjoint solve)
__global__ void k_set_rhs_adjoint(const RepDev *reps, const int *body_rep, int nb, const double *Ubar, double *b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nb) return;
    int p = t / 6, k = t % 6;
    const RepDev &R = reps[body_rep[p]];
    b[R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0) + k] = R.dV * Ubar[t];
}

void launch_set_rhs_adjoint(Ctx &c, const double *Ubar, double *b) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_set_rhs_adjoint, dim3((6 * c.nb + 255) / 256), dim3(256), 0, c.stream, c.d_reps,
                       c.d_body_rep, c.nb, Ubar, b);
}

}  // namespace rb

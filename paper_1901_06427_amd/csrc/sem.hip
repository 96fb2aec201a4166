// Kernels of one Split-Euler-Maruyama step (paper Sec. IV, Algorithm 1), with the
// drift signs read from eqs. D1-D4 and the correctly signed chain rule of dN:
//   W^FT_p = kT [W^f / L_p ; W^tau],  Q+- = (q +- (delta/2) L_p W^f, Rotate(theta, +-(delta/2) W^tau)),
//   D^KT = (1/delta)[K^T(Q+) - K^T(Q-)] lambda^R,  D^K = (1/delta)[K(Q+) - K(Q-)] U^R,
//   D^J = (1/delta)[J(Q+) - J(Q-)] v^R,  D^S = J(Q) v#,
//   step-6 system: force F - D^KT, slip  slip + D^K - D^J - D^S.
// Random numbers: Philox4x32-10 stream 0 holds 6 normals per body (W^f then W^tau),
// replica r uses seed + r.
#include "common.h"

namespace rb {

__global__ void k_body_rfd(const RepDev *reps, const int *body_rep, const double *body_len, int nb, const double *q,
                           const double *theta, double kT, double delta, uint64_t seed, uint64_t step, double *Wf,
                           double *Wt, double *WFT, double *qp, double *thp, double *qm, double *thm) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    int r = body_rep[p];
    const RepDev &R = reps[r];
    uint64_t rseed = seed + (uint64_t)r;
    uint64_t base = 6ULL * (uint64_t)(p - R.b0);
    double wf[3], wt[3];
    for (int k = 0; k < 3; ++k) {
        wf[k] = philox_normal(rseed, 0u, step, base + k);
        wt[k] = philox_normal(rseed, 0u, step, base + 3 + k);
    }
    double Lp = body_len[p];
    for (int k = 0; k < 3; ++k) {
        Wf[3 * p + k] = wf[k];
        Wt[3 * p + k] = wt[k];
        WFT[6 * p + k] = kT * wf[k] / Lp;
        WFT[6 * p + 3 + k] = kT * wt[k];
        double dq = 0.5 * delta * Lp * wf[k];
        qp[3 * p + k] = q[3 * p + k] + dq;
        qm[3 * p + k] = q[3 * p + k] - dq;
    }
    double php[3] = {0.5 * delta * wt[0], 0.5 * delta * wt[1], 0.5 * delta * wt[2]};
    double phm[3] = {-php[0], -php[1], -php[2]};
    quat_rotate(theta + 4 * p, php, thp + 4 * p);
    quat_rotate(theta + 4 * p, phm, thm + 4 * p);
}

void launch_body_rfd(Ctx &c, double kT, double delta, uint64_t seed, uint64_t step, const double *q,
                     const double *theta) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_body_rfd, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_reps, c.d_body_rep,
                       c.d_body_len, c.nb, q, theta, kT, delta, seed, step, c.Wf, c.Wt, c.WFT, c.q_buf[0],
                       c.th_buf[0], c.q_buf[1], c.th_buf[1]);
}

// slip_acc[m, c] = D^K - D^J  at every marker (Q+ in ms_p, Q- in ms_m; xR holds v^R and U^R).
template <int W>
__global__ void k_rfd_markers(const RepDev *reps, const int *marker_body, const int *body_rep, int nm,
                              const double *wcp, const int *icp, const double *dp, const double *wcm, const int *icm,
                              const double *dm, const double *__restrict__ xR, double inv_delta,
                              double *__restrict__ slip_acc) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nm) return;
    int m = t / 3, c = t % 3;
    int p = marker_body[m];
    const RepDev &R = reps[body_rep[p]];
    const double *UR = xR + R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0);
    // D^K: (omega^R x d+) - (omega^R x d-) ; the translation cancels exactly
    const double *a = dp + 3 * m, *b = dm + 3 * m;
    double kp[3] = {UR[4] * a[2] - UR[5] * a[1], UR[5] * a[0] - UR[3] * a[2], UR[3] * a[1] - UR[4] * a[0]};
    double km[3] = {UR[4] * b[2] - UR[5] * b[1], UR[5] * b[0] - UR[3] * b[2], UR[3] * b[1] - UR[4] * b[0]};
    double DK = ((UR[c] + kp[c]) - (UR[c] + km[c])) * inv_delta;
    const double *u = xR + R.off + c * R.N;
    double DJ = (interp_cached<W>(R, wcp, icp, m, c, u) - interp_cached<W>(R, wcm, icm, m, c, u)) * inv_delta;
    slip_acc[t] = DK - DJ;
}

// F'_p = FT_p - D^KT_p
__global__ void k_rfd_bodies(const RepDev *reps, const int *body_rep, const int *body_off, int nb, const double *dp,
                             const double *dm, const double *__restrict__ xR, double inv_delta, const double *FT,
                             double *Fp) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    const RepDev &R = reps[body_rep[p]];
    double sp[6] = {0, 0, 0, 0, 0, 0}, sm[6] = {0, 0, 0, 0, 0, 0};
    for (int m = body_off[p]; m < body_off[p + 1]; ++m) {
        const double *l = xR + R.off + 4 * R.N + 3LL * (m - R.m0);
        const double *a = dp + 3 * m, *b = dm + 3 * m;
        for (int k = 0; k < 3; ++k) { sp[k] += l[k]; sm[k] += l[k]; }
        sp[3] += a[1] * l[2] - a[2] * l[1]; sp[4] += a[2] * l[0] - a[0] * l[2]; sp[5] += a[0] * l[1] - a[1] * l[0];
        sm[3] += b[1] * l[2] - b[2] * l[1]; sm[4] += b[2] * l[0] - b[0] * l[2]; sm[5] += b[0] * l[1] - b[1] * l[0];
    }
    for (int k = 0; k < 6; ++k) Fp[6 * p + k] = (FT ? FT[6 * p + k] : 0.0) - (sp[k] - sm[k]) * inv_delta;
}

void launch_rfd_terms(Ctx &c, double delta) {
    if (c.nm == 0) return;
    double inv = 1.0 / delta;
    hipLaunchKernelGGL(c.kw == 6 ? k_rfd_markers<6> : k_rfd_markers<4>, dim3((3 * c.nm + 255) / 256), dim3(256), 0, c.stream, c.d_reps,
                       c.d_marker_body, c.d_body_rep, c.nm, c.ms[1].wc, c.ms[1].ic, c.ms[1].d, c.ms[2].wc,
                       c.ms[2].ic, c.ms[2].d, c.xR, inv, c.slip_acc);
}

void launch_rfd_forces(Ctx &c, double delta, const double *FT) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_rfd_bodies, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_reps, c.d_body_rep,
                       c.d_body_off, c.nb, c.ms[1].d, c.ms[2].d, c.xR, 1.0 / delta, FT, c.Fp);
}

// b_lambda[m] = -(slip + slip_acc - D^S) + J_bc, with D^S = J(Q^n) v#  (v# in xS).
template <int W>
__global__ void k_sem_rhs_lambda(const RepDev *reps, const int *marker_body, const int *body_rep, int nm,
                                 const double *wc, const int *ic, const double *slip, const double *slip_acc,
                                 const double *__restrict__ xS, double *__restrict__ b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nm) return;
    int m = t / 3, c = t % 3;
    const RepDev &R = reps[body_rep[marker_body[m]]];
    double DS = interp_cached<W>(R, wc, ic, m, c, xS + R.off + c * R.N);
    double s2 = slip_acc[t] - DS + (slip ? slip[t] : 0.0);
    b[R.off + 4 * R.N + 3LL * (m - R.m0) + c] = -s2;
}

void launch_sem_rhs_lambda(Ctx &c, const double *slip, double *b) {
    if (c.nm == 0) return;
    hipLaunchKernelGGL(c.kw == 6 ? k_sem_rhs_lambda<6> : k_sem_rhs_lambda<4>, dim3((3 * c.nm + 255) / 256), dim3(256), 0, c.stream, c.d_reps,
                       c.d_marker_body, c.d_body_rep, c.nm, c.ms[0].wc, c.ms[0].ic, slip, c.slip_acc, c.xS, b);
}

// b_U[p] = F'_p
__global__ void k_set_rhs_U(const RepDev *reps, const int *body_rep, int nb, const double *Fp, double *b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nb) return;
    int p = t / 6, k = t % 6;
    const RepDev &R = reps[body_rep[p]];
    b[R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0) + k] = Fp[t];
}

void launch_set_rhs_U(Ctx &c, const double *Fp, double *b) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_set_rhs_U, dim3((6 * c.nb + 255) / 256), dim3(256), 0, c.stream, c.d_reps, c.d_body_rep,
                       c.nb, Fp, b);
}

// q_new = q + dt u, theta_new = Rotate(theta, dt omega) from the solution x.
__global__ void k_update_positions(const RepDev *reps, const int *body_rep, int nb, const double *q,
                                   const double *theta, const double *__restrict__ x, double dt, double *qn,
                                   double *thn) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    const RepDev &R = reps[body_rep[p]];
    const double *U = x + R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0);
    for (int k = 0; k < 3; ++k) qn[3 * p + k] = q[3 * p + k] + dt * U[k];
    double ph[3] = {dt * U[3], dt * U[4], dt * U[5]};
    quat_rotate(theta + 4 * p, ph, thn + 4 * p);
}

void launch_update_positions(Ctx &c, const double *q, const double *theta, const double *x, double dt) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_update_positions, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_reps, c.d_body_rep,
                       c.nb, q, theta, x, dt, c.q_buf[2], c.th_buf[2]);
}

// Stage update of the second-order variants: U_c = U^n + w (U_det* - U_det^n), then
// q_new = q + dt u_c and theta_new = Rotate(theta, dt omega_c) into q_buf[2], th_buf[2]
// (w = 0 gives the predictor's move by U^n itself).
__global__ void k_rk2_update(int nb, const double *q, const double *theta, const double *Uem, const double *Ud0,
                             const double *Ud1, double w, double dt, double *Uc, double *qn, double *thn) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    double u[6];
    for (int k = 0; k < 6; ++k) {
        u[k] = w == 0.0 ? Uem[6 * p + k] : Uem[6 * p + k] + w * (Ud1[6 * p + k] - Ud0[6 * p + k]);
        if (Uc) Uc[6 * p + k] = u[k];
    }
    for (int k = 0; k < 3; ++k) qn[3 * p + k] = q[3 * p + k] + dt * u[k];
    double ph[3] = {dt * u[3], dt * u[4], dt * u[5]};
    quat_rotate(theta + 4 * p, ph, thn + 4 * p);
}

void launch_rk2_update(Ctx &c, const double *q, const double *theta, const double *Uem, const double *Ud0,
                       const double *Ud1, double w, double dt, double *Uc) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_rk2_update, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.nb, q, theta, Uem, Ud0, Ud1,
                       w, dt, Uc, c.q_buf[2], c.th_buf[2]);
}

// Rejection by body-centre distance (per replica flag).
__global__ void k_body_distance(const RepDev *reps, const int *body_rep, int nb, const double *qn, double dmin,
                                int *rep_flags) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    int r = body_rep[p];
    const RepDev &R = reps[r];
    for (int o = R.b0; o < R.b0 + R.nb; ++o) {
        if (o == p) continue;
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double d = qn[3 * p + k] - qn[3 * o + k];
            if (R.bc[k] == RBFIB_PERIODIC) {
                double L = R.n[k] * R.h;
                d -= L * nearbyint(d / L);
            }
            d2 += d * d;
        }
        if (d2 < dmin * dmin) atomicOr(&rep_flags[r], 2);
    }
}

void launch_body_distance(Ctx &c, double dmin) {
    if (c.nb == 0 || !(dmin > 0.0)) return;
    hipLaunchKernelGGL(k_body_distance, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_reps, c.d_body_rep, c.nb,
                       c.q_buf[2], dmin, c.d_flags);
}

// Accept the new configuration of replicas whose flag is clear.
__global__ void k_commit(const int *body_rep, int nb, const int *rep_flags, const double *qn, const double *thn,
                         double *q, double *theta) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nb) return;
    if (rep_flags[body_rep[p]]) return;
    for (int k = 0; k < 3; ++k) q[3 * p + k] = qn[3 * p + k];
    for (int k = 0; k < 4; ++k) theta[4 * p + k] = thn[4 * p + k];
}

void launch_commit_positions(Ctx &c, double *q, double *theta) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_commit, dim3((c.nb + 63) / 64), dim3(64), 0, c.stream, c.d_body_rep, c.nb, c.d_flags,
                       c.q_buf[2], c.th_buf[2], q, theta);
}

}  // namespace rb

// Fused multigrid level kernels (V(2,2) damped Jacobi), marching along z.
//
// A workgroup owns an MGF_OX x MGF_OY x MGF_ZC block of fine points of one
// component and walks its z planes in order, keeping a few (x, y) planes with a
// two-point halo in LDS:
//
// k_mg_down: plane t   <- b and the first sweep from zero, x1 = w b
//            plane t-1 <- second sweep x2 from the x1 planes t-2 .. t
//            plane t-2 <- residual r = b - A x2; x2 of owned points to HBM
//            then every coarse plane whose fine planes are complete is
//            restricted (full weighting on the face-normal axis, pairs on the
//            cell axes) and written.
// k_mg_up:   plane t   <- x + P x_coarse
//            plane t-1 <- first sweep; plane t-2 <- second sweep, written.
//
// Per level: b read once and x written once going down, x, b read and x written
// once going up, instead of six separate passes.  The operator, boundary rules,
// transfer weights and the rounding of every operation are those of the separate
// kernels in grid.hip (shared helpers in common.h), so the V-cycle output is
// bit-identical.
#include "common.h"

namespace rb {

#define MGF_PLANE ((MGF_OX + 5) * (MGF_OY + 5))
#define MGF_NS ((MGF_PLANE + 255) / 256)

__device__ __forceinline__ int wrap_axis(int g, int n) {
    if (g < 0) g += n;
    if (g < 0) g += n;
    if (g >= n) g -= n;
    if (g >= n) g -= n;
    return g;
}

// Per-thread description of its (x, y) plane positions.
template <typename T>
struct PlaneSlots {
    int p[MGF_NS];       // plane index, -1 if unused
    int l0[MGF_NS], l1[MGF_NS];
    int g0[MGF_NS], g1[MGF_NS];   // wrapped coordinates
    int gxy[MGF_NS];     // g0 + n0 g1
    bool in[MGF_NS];     // (x, y) inside the domain
    bool pin[MGF_NS];    // pinned through the x or y coordinate
    int kinds[MGF_NS];   // 2 bits each: x-, x+, y-, y+
    T dxy[MGF_NS];       // diagonal terms of x and y
};

template <typename T>
__device__ __forceinline__ void make_slots(PlaneSlots<T> &S, int PX, int PY, int px0, int py0, const LevDev &F,
                                           const RepDev &R, int comp) {
#pragma unroll
    for (int k = 0; k < MGF_NS; ++k) {
        const int p = threadIdx.x + k * 256;
        S.p[k] = p < PX * PY ? p : -1;
        const int l1 = p / PX, l0 = p - l1 * PX;
        S.l0[k] = l0;
        S.l1[k] = l1;
        int g0 = px0 + l0, g1 = py0 + l1;
        bool in0 = R.bc[0] == RBFIB_PERIODIC || (g0 >= 0 && g0 < F.n[0]);
        bool in1 = R.bc[1] == RBFIB_PERIODIC || (g1 >= 0 && g1 < F.n[1]);
        if (R.bc[0] == RBFIB_PERIODIC) g0 = wrap_axis(g0, F.n[0]);
        if (R.bc[1] == RBFIB_PERIODIC) g1 = wrap_axis(g1, F.n[1]);
        S.in[k] = in0 && in1;
        S.g0[k] = g0;
        S.g1[k] = g1;
        S.gxy[k] = S.in[k] ? g0 + F.n[0] * g1 : 0;
        S.pin[k] = (comp == 0 && R.bc[0] != RBFIB_PERIODIC && g0 == 0) || (comp == 1 && R.bc[1] != RBFIB_PERIODIC && g1 == 0);
        S.kinds[k] = nbr_kind(g0, -1, F.n[0], R.bc[0], 0, comp) | (nbr_kind(g0, +1, F.n[0], R.bc[0], 0, comp) << 2) |
                     (nbr_kind(g1, -1, F.n[1], R.bc[1], 1, comp) << 4) |
                     (nbr_kind(g1, +1, F.n[1], R.bc[1], 1, comp) << 6);
        S.dxy[k] = fmad(diag_axis<T>(comp, 1, g1, F.n[1], R.bc[1]), (T)F.inv_h2[1],
                        fmad(diag_axis<T>(comp, 0, g0, F.n[0], R.bc[0]), (T)F.inv_h2[0], (T)0));
    }
}

// One z plane of a marching block: unwrapped z, wrapped index, membership, rules.
struct ZPlane {
    int z, gz;
    bool in, pin;
    int km, kp;
};

__device__ __forceinline__ ZPlane zplane(int z, const LevDev &F, const RepDev &R, int comp) {
    ZPlane P;
    P.z = z;
    if (R.bc[2] == RBFIB_PERIODIC) { P.in = true; P.gz = wrap_axis(z, F.n[2]); }
    else { P.in = z >= 0 && z < F.n[2]; P.gz = P.in ? z : 0; }
    P.pin = comp == 2 && R.bc[2] != RBFIB_PERIODIC && P.gz == 0;
    P.km = nbr_kind(P.gz, -1, F.n[2], R.bc[2], 2, comp);
    P.kp = nbr_kind(P.gz, +1, F.n[2], R.bc[2], 2, comp);
    return P;
}

// 7-point Laplacian at plane position p of plane slot c (neighbour planes cm, cp),
// same association as lap_point in grid.hip.
template <typename T>
__device__ __forceinline__ T lap_planes(const T (*A)[MGF_PLANE], int cm, int c, int cp, int p, int PX, int kinds,
                                        const ZPlane &Z, const LevDev &F) {
    const T self = A[c][p];
    T acc = lap_acc<T>(pick<T>((kinds >> 2) & 3, A[c][p + 1], self), self, pick<T>(kinds & 3, A[c][p - 1], self),
                       (T)F.inv_h2[0], (T)0);
    acc = lap_acc<T>(pick<T>((kinds >> 6) & 3, A[c][p + PX], self), self,
                     pick<T>((kinds >> 4) & 3, A[c][p - PX], self), (T)F.inv_h2[1], acc);
    acc = lap_acc<T>(pick<T>(Z.kp, A[cp][p], self), self, pick<T>(Z.km, A[cm][p], self), (T)F.inv_h2[2], acc);
    return acc;
}

// Tile of the fused kernels: tile index -> owned fine block [lo, hi) per axis.
__device__ __forceinline__ void mg_tile(long long t, const LevDev &F, int lo[3], int hi[3]) {
    const int nt0 = (F.n[0] + MGF_OX - 1) / MGF_OX, nt1 = (F.n[1] + MGF_OY - 1) / MGF_OY;
    const int t0 = (int)(t % nt0);
    t /= nt0;
    const int t1 = (int)(t % nt1);
    const int t2 = (int)(t / nt1);
    lo[0] = t0 * MGF_OX; lo[1] = t1 * MGF_OY; lo[2] = t2 * MGF_ZC;
    hi[0] = min(lo[0] + MGF_OX, F.n[0]);
    hi[1] = min(lo[1] + MGF_OY, F.n[1]);
    hi[2] = min(lo[2] + MGF_ZC, F.n[2]);
}

// ------------------------------------------------------------------ down
template <typename T>
__global__ __launch_bounds__(256) void k_mg_down(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                  int lev, int c0, const T *bpool, T *__restrict__ xpool, T *bcpool,
                                                  double omega1, double omega2, const int *__restrict__ mask) {
    __shared__ T sB[3][MGF_PLANE];
    __shared__ T sW[3][MGF_PLANE];
    __shared__ T sX1[3][MGF_PLANE];
    __shared__ T sX2[3][MGF_PLANE];
    __shared__ T sR[3][MGF_PLANE];
    const BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    const T om1 = (T)omega1, om2 = (T)omega2;
    int lo[3], hi[3], fr[3];
    bool crs[3];
    mg_tile(be.start, F, lo, hi);
    for (int a = 0; a < 3; ++a) {
        crs[a] = F.n[a] != C.n[a];
        fr[a] = (crs[a] && a == comp) ? 1 : 0;   // the residual also covers face 2I-1 of the first coarse face
    }
    const int PX = hi[0] - lo[0] + fr[0] + 4, PY = hi[1] - lo[1] + fr[1] + 4;
    const int px0 = lo[0] - fr[0] - 2, py0 = lo[1] - fr[1] - 2;
    const int Z0 = lo[2] - fr[2] - 2;
    const int NZ = hi[2] - lo[2] + fr[2];        // residual planes
    PlaneSlots<T> S;
    make_slots<T>(S, PX, PY, px0, py0, F, R, comp);
    const T *b = bpool + F.off + comp * F.N;
    T *x = xpool + F.off + comp * F.N;
    T *bc = bcpool + C.off + comp * C.N;
    const int n01 = F.n[0] * F.n[1];
    // coarse points owned by this block
    int clo[3], chi[3];
    for (int a = 0; a < 3; ++a) {
        clo[a] = crs[a] ? lo[a] / 2 : lo[a];
        chi[a] = crs[a] ? hi[a] / 2 : hi[a];
    }
    const int cex = chi[0] - clo[0], cey = chi[1] - clo[1];

    // b of the next plane is loaded one iteration ahead, so that its latency
    // overlaps the sweeps of the current planes (the barriers wait on LDS only)
    T nb[MGF_NS];
    auto fetch = [&](int t) {
        const ZPlane Z = zplane(Z0 + t, F, R, comp);
#pragma unroll
        for (int k = 0; k < MGF_NS; ++k)
            nb[k] = (S.p[k] >= 0 && S.in[k] && Z.in && !S.pin[k] && !Z.pin) ? b[S.gxy[k] + n01 * Z.gz] : (T)0;
    };
    fetch(0);
    for (int t = 0; t <= NZ + 3; ++t) {
        // plane t: b, weight and the first sweep from zero
        {
            const ZPlane Z = zplane(Z0 + t, F, R, comp);
            const int c = t % 3;
            const T dz = (T)F.inv_h2[2];
            const T daz = diag_axis<T>(comp, 2, Z.gz, F.n[2], R.bc[2]);
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0) continue;
                T d = (T)0, x1 = (T)0;
                if (S.in[k] && Z.in && !S.pin[k] && !Z.pin) {
                    d = fmad(daz, dz, S.dxy[k]);
                    x1 = nb[k] * jacobi_w<T>(om1, s, d);
                }
                sB[c][S.p[k]] = nb[k];
                sW[c][S.p[k]] = d;
                sX1[c][S.p[k]] = x1;
            }
        }
        if (t + 1 <= NZ + 3) fetch(t + 1);
        __syncthreads();
        // plane t-1: second sweep
        if (t >= 2) {
            const int tb = t - 1;
            const ZPlane Z = zplane(Z0 + tb, F, R, comp);
            const int c = tb % 3, cm = (tb + 2) % 3, cp = t % 3;
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0 || S.l0[k] < 1 || S.l0[k] > PX - 2 || S.l1[k] < 1 || S.l1[k] > PY - 2) continue;
                T x2 = (T)0;
                if (S.in[k] && Z.in && !S.pin[k] && !Z.pin) {
                    const T lap = lap_planes<T>(sX1, cm, c, cp, S.p[k], PX, S.kinds[k], Z, F);
                    x2 = jacobi_step<T>(sX1[c][S.p[k]], sB[c][S.p[k]], s, lap, jacobi_w<T>(om2, s, sW[c][S.p[k]]));
                }
                sX2[c][S.p[k]] = x2;
            }
        }
        __syncthreads();
        // plane t-2: residual; owned x written
        const int tc = t - 2;
        if (t >= 4) {
            const ZPlane Z = zplane(Z0 + tc, F, R, comp);
            const int c = tc % 3, cm = (tc + 2) % 3, cp = (tc + 1) % 3;
            const bool zown = Z.z >= lo[2] && Z.z < hi[2];
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0 || S.l0[k] < 2 || S.l0[k] > PX - 3 || S.l1[k] < 2 || S.l1[k] > PY - 3) continue;
                T r = (T)0;
                if (S.in[k] && Z.in) {
                    const int ux = px0 + S.l0[k], uy = py0 + S.l1[k];
                    if (zown && ux >= lo[0] && ux < hi[0] && uy >= lo[1] && uy < hi[1])
                        x[S.gxy[k] + n01 * Z.gz] = sX2[c][S.p[k]];
                    if (!S.pin[k] && !Z.pin) {
                        const T lap = lap_planes<T>(sX2, cm, c, cp, S.p[k], PX, S.kinds[k], Z, F);
                        r = mg_residual<T>(sB[c][S.p[k]], s, lap);
                    }
                }
                sR[c][S.p[k]] = r;
            }
        }
        __syncthreads();
        // coarse plane K whose fine residual planes are complete
        if (t >= 4) {
            const int z = Z0 + tc;              // unwrapped fine z of the newest residual plane
            int K = -1, nk = 1, zf = tc;        // zf: relative index of the first fine plane
            if (!crs[2]) {
                if (z >= lo[2] && z < hi[2]) K = z;
            } else if ((z & 1) && z - 1 >= lo[2] && z - 1 < hi[2]) {
                K = (z - 1) >> 1;
                nk = fr[2] ? 3 : 2;
                zf = tc - nk + 1;
            }
            if (K >= 0) {
                const int c01 = C.n[0] * C.n[1];
                for (int q = threadIdx.x; q < cex * cey; q += blockDim.x) {
                    const int J = clo[1] + q / cex, I = clo[0] + q % cex;
                    T *out = bc + I + C.n[0] * J + c01 * K;
                    const int ci[3] = {I, J, K};
                    if (comp < 3 && R.bc[comp] != RBFIB_PERIODIC && ci[comp] == 0) { *out = (T)0; continue; }
                    const int fb0 = (crs[0] ? 2 * I - fr[0] : I) - px0;
                    const int fb1 = (crs[1] ? 2 * J - fr[1] : J) - py0;
                    const int nx = !crs[0] ? 1 : (fr[0] ? 3 : 2), ny = !crs[1] ? 1 : (fr[1] ? 3 : 2);
                    T acc = (T)0;
                    for (int kk = 0; kk < nk; ++kk) {
                        const int cz = (zf + kk) % 3;
                        const T wz = restrict_weight<T>(crs[2], fr[2] != 0, kk);
                        for (int jj = 0; jj < ny; ++jj) {
                            const T wy = restrict_weight<T>(crs[1], fr[1] != 0, jj);
                            for (int ii = 0; ii < nx; ++ii) {
                                const T wx = restrict_weight<T>(crs[0], fr[0] != 0, ii);
                                acc = fmad(wx * wy * wz, sR[cz][fb0 + ii + PX * (fb1 + jj)], acc);
                            }
                        }
                    }
                    *out = acc;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ up
template <typename T>
__global__ __launch_bounds__(256) void k_mg_up(const RepDev *reps, const LevDev *levs, const BlockEnt *tab, int lev,
                                                int c0, const T *__restrict__ bpool, const T *__restrict__ xinpool,
                                                const T *__restrict__ xcpool, T *__restrict__ xoutpool, double omega1,
                                                double omega2, const int *__restrict__ mask) {
    __shared__ T sB[3][MGF_PLANE];
    __shared__ T sW[3][MGF_PLANE];
    __shared__ T sXP[3][MGF_PLANE];
    __shared__ T sXS[3][MGF_PLANE];
    const BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    const T om1 = (T)omega1, om2 = (T)omega2;
    int lo[3], hi[3];
    mg_tile(be.start, F, lo, hi);
    const int PX = hi[0] - lo[0] + 4, PY = hi[1] - lo[1] + 4;
    const int px0 = lo[0] - 2, py0 = lo[1] - 2;
    const int Z0 = lo[2] - 2;
    const int NZ = hi[2] - lo[2];
    PlaneSlots<T> S;
    make_slots<T>(S, PX, PY, px0, py0, F, R, comp);
    const T *b = bpool + F.off + comp * F.N;
    const T *xin = xinpool + F.off + comp * F.N;
    const T *xc = xcpool + C.off + comp * C.N;
    T *xo = xoutpool + F.off + comp * F.N;
    const int n01 = F.n[0] * F.n[1];
    const long long c01 = (long long)C.n[0] * C.n[1];

    // b, x and the (up to 8) coarse values of the next plane are loaded one
    // iteration ahead; P x_c is summed in the order of prolong_at
    T nb[MGF_NS], nx[MGF_NS], ncv[MGF_NS][8];
    auto fetch = [&](int t) {
        const ZPlane Z = zplane(Z0 + t, F, R, comp);
        const ProlongAxis<T> pz = prolong_axis<T>(Z.gz, F.n[2], C.n[2], R.bc[2], comp == 2, comp);
#pragma unroll
        for (int k = 0; k < MGF_NS; ++k) {
            const bool ok = S.p[k] >= 0 && S.in[k] && Z.in && !S.pin[k] && !Z.pin;
            const int gi = S.gxy[k] + n01 * Z.gz;
            nb[k] = ok ? b[gi] : (T)0;
            nx[k] = ok ? xin[gi] : (T)0;
            const ProlongAxis<T> px = prolong_axis<T>(S.g0[k], F.n[0], C.n[0], R.bc[0], comp == 0, comp);
            const ProlongAxis<T> py = prolong_axis<T>(S.g1[k], F.n[1], C.n[1], R.bc[1], comp == 1, comp);
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii) {
                        const bool use = ok && kk < pz.cnt && jj < py.cnt && ii < px.cnt;
                        const long long ci = (ii ? px.i1 : px.i0) + (long long)C.n[0] * (jj ? py.i1 : py.i0) +
                                             c01 * (kk ? pz.i1 : pz.i0);
                        ncv[k][kk * 4 + jj * 2 + ii] = use ? xc[ci] : (T)0;
                    }
        }
    };
    fetch(0);
    for (int t = 0; t <= NZ + 3; ++t) {
        // plane t: x + P x_c, b and weight
        {
            const ZPlane Z = zplane(Z0 + t, F, R, comp);
            const int c = t % 3;
            const T daz = diag_axis<T>(comp, 2, Z.gz, F.n[2], R.bc[2]);
            const ProlongAxis<T> pz = prolong_axis<T>(Z.gz, F.n[2], C.n[2], R.bc[2], comp == 2, comp);
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0) continue;
                T d = (T)0, v = (T)0;
                if (S.in[k] && Z.in && !S.pin[k] && !Z.pin) {
                    d = fmad(daz, (T)F.inv_h2[2], S.dxy[k]);
                    const ProlongAxis<T> px = prolong_axis<T>(S.g0[k], F.n[0], C.n[0], R.bc[0], comp == 0, comp);
                    const ProlongAxis<T> py = prolong_axis<T>(S.g1[k], F.n[1], C.n[1], R.bc[1], comp == 1, comp);
                    T acc = (T)0;
#pragma unroll
                    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                            for (int ii = 0; ii < 2; ++ii)
                                if (kk < pz.cnt && jj < py.cnt && ii < px.cnt)
                                    acc = fmad((ii ? px.w1 : px.w0) * (jj ? py.w1 : py.w0) * (kk ? pz.w1 : pz.w0),
                                               ncv[k][kk * 4 + jj * 2 + ii], acc);
                    v = nx[k] + acc;
                }
                sB[c][S.p[k]] = nb[k];
                sW[c][S.p[k]] = d;
                sXP[c][S.p[k]] = v;
            }
        }
        if (t + 1 <= NZ + 3) fetch(t + 1);
        __syncthreads();
        // plane t-1: first sweep
        if (t >= 2) {
            const int tb = t - 1;
            const ZPlane Z = zplane(Z0 + tb, F, R, comp);
            const int c = tb % 3, cm = (tb + 2) % 3, cp = t % 3;
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0 || S.l0[k] < 1 || S.l0[k] > PX - 2 || S.l1[k] < 1 || S.l1[k] > PY - 2) continue;
                T v = (T)0;
                if (S.in[k] && Z.in && !S.pin[k] && !Z.pin) {
                    const T lap = lap_planes<T>(sXP, cm, c, cp, S.p[k], PX, S.kinds[k], Z, F);
                    v = jacobi_step<T>(sXP[c][S.p[k]], sB[c][S.p[k]], s, lap, jacobi_w<T>(om1, s, sW[c][S.p[k]]));
                }
                sXS[c][S.p[k]] = v;
            }
        }
        __syncthreads();
        // plane t-2: second sweep, written
        if (t >= 4) {
            const int tc = t - 2;
            const ZPlane Z = zplane(Z0 + tc, F, R, comp);
            const int c = tc % 3, cm = (tc + 2) % 3, cp = (tc + 1) % 3;
#pragma unroll
            for (int k = 0; k < MGF_NS; ++k) {
                if (S.p[k] < 0 || S.l0[k] < 2 || S.l0[k] > PX - 3 || S.l1[k] < 2 || S.l1[k] > PY - 3) continue;
                if (!S.in[k] || !Z.in) continue;
                const int gi = S.gxy[k] + n01 * Z.gz;
                if (S.pin[k] || Z.pin) { xo[gi] = (T)0; continue; }
                const T lap = lap_planes<T>(sXS, cm, c, cp, S.p[k], PX, S.kinds[k], Z, F);
                xo[gi] = jacobi_step<T>(sXS[c][S.p[k]], sB[c][S.p[k]], s, lap, jacobi_w<T>(om2, s, sW[c][S.p[k]]));
            }
        }
        __syncthreads();
    }
}

template <typename T>
void launch_mg_down(Ctx &c, int lev, int c0, int nc, const T *b, T *x, double omega1, double omega2) {
    int n = c.n_tab_mg[lev];
    if (n == 0) return;
    hipLaunchKernelGGL(k_mg_down<T>, dim3(n, nc), dim3(256), 0, c.stream, c.d_reps, c.d_levs, c.d_tab_mg[lev], lev,
                       c0, b, x, (T *)b, omega1, omega2, c.mask);
    HIP_OK(hipGetLastError());
}

template <typename T>
void launch_mg_up(Ctx &c, int lev, int c0, int nc, const T *b, const T *xin, const T *xc, T *xout, double omega1,
                  double omega2) {
    int n = c.n_tab_mg[lev];
    if (n == 0) return;
    hipLaunchKernelGGL(k_mg_up<T>, dim3(n, nc), dim3(256), 0, c.stream, c.d_reps, c.d_levs, c.d_tab_mg[lev], lev, c0,
                       b, xin, xc, xout, omega1, omega2, c.mask);
    HIP_OK(hipGetLastError());
}

template void launch_mg_down<float>(Ctx &, int, int, int, const float *, float *, double, double);
template void launch_mg_down<double>(Ctx &, int, int, int, const double *, double *, double, double);
template void launch_mg_up<float>(Ctx &, int, int, int, const float *, const float *, const float *, float *, double,
                                  double);
template void launch_mg_up<double>(Ctx &, int, int, int, const double *, const double *, const double *, double *,
                                   double, double);

}  // namespace rb

// Staggered-grid kernels: the fused saddle-point fluid apply (-eta Lm v + G pi, -D v),
// the geometric-multigrid pieces of the Stokes preconditioner (damped Jacobi,
// restriction, prolongation, dense coarsest solve, projection step), the
// fluctuating-stress forcing DT W and the sliding-wall terms.
//
// Discretisation (paper Sec. III.A): velocity on faces, pressure at cell centres,
// G = -D^*, Lm = DT GT; on a wall axis the normal-velocity wall faces are not
// unknowns and tangential ghosts are u_g = 2 U_w - u at a no-slip wall (the
// homogeneous operator uses U_w = 0) and u_g = u at a free-slip wall.  Every kernel is one thread per grid point, x fastest, so that a
// wavefront reads 64 consecutive doubles of each field.
#include "common.h"

namespace rb {

// Value of field u (component c, or 3 = pressure) at the neighbour of (i,j,k)
// along axis a in direction d (+1/-1), with the boundary rule of the operator.
template <typename T>
__device__ __forceinline__ T nbr(const T *u, int c, int a, int d, int idx[3], const int n[3], const int bc[3],
                                 T self, long long lin, long long stride) {
    int p = idx[a] + d;
    if (bc[a] == RBFIB_PERIODIC) {
        if (p < 0) return u[lin + (long long)(n[a] - 1) * stride];
        if (p >= n[a]) return u[lin - (long long)(n[a] - 1) * stride];
        return u[lin + d * stride];
    }
    if (a == c) {                       // face-normal: wall faces are zero
        if (p <= 0 || p >= n[a]) return (T)0;
        return u[lin + d * stride];
    }
    if (p < 0 || p >= n[a]) return even_ghost(c, bc[a]) ? self : -self;   // even / odd ghost
    return u[lin + d * stride];
}

// sum_a (u(+a) - 2u + u(-a)) * inv_h2[a]  and its diagonal coefficient.
template <typename T>
__device__ __forceinline__ T lap_point(const T *u, int c, int idx[3], const int n[3], const int bc[3],
                                       const double ih2[3], long long lin, T &diag) {
    T self = u[lin];
    T acc = (T)0;
    T dg = (T)0;
    long long stride = 1;
    for (int a = 0; a < 3; ++a) {
        T up = nbr(u, c, a, +1, idx, n, bc, self, lin, stride);
        T um = nbr(u, c, a, -1, idx, n, bc, self, lin, stride);
        acc = lap_acc<T>(up, self, um, (T)ih2[a], acc);
        dg = fmad(diag_axis<T>(c, a, idx[a], n[a], bc[a]), (T)ih2[a], dg);
        stride *= n[a];
    }
    diag = dg;
    return acc;
}

__device__ __forceinline__ bool pinned(int c, const int idx[3], const int bc[3]) {
    return c < 3 && bc[c] != RBFIB_PERIODIC && idx[c] == 0;
}

__device__ __forceinline__ void unlin(long long lin, const RepDev &R, int idx[3]) {
    split_index(lin, R.n[0], R.n[0] * R.n[1], R.inv_n0, R.inv_n01, idx);
}

__device__ __forceinline__ void unlin(long long lin, const LevDev &L, int idx[3]) {
    split_index(lin, L.n[0], L.n[0] * L.n[1], L.inv_n0, L.inv_n01, idx);
}

// ------------------------------------------------------------------ fused fluid apply
// y_c = -eta Lm_c v + (G pi)_c for c = x, y, z;  y_pi = -(D v).  Pinned slots -> 0.
// The three momentum rows and the divergence of one cell from its gathered values:
// self[c] = v_c of the cell, nb[c][2a] / nb[c][2a+1] its -e_a / +e_a neighbours (rule
// kd), pm[c] the pressure at -e_c, pc the cell's.  Explicit fused multiply-adds, so
// both gather paths below round identically.
__device__ __forceinline__ void apply_cell(const RepDev &R, const double self[3], const double nb[3][6],
                                           const double pm[3], double pc, const int kd[3][6], const bool pin[3],
                                           double out[4]) {
    const double ih = R.inv_h, ih2 = R.inv_h * R.inv_h;
    double div = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double lap = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            lap = lap_acc<double>(pick<double>(kd[c][2 * a + 1], nb[c][2 * a + 1], self[c]), self[c],
                                  pick<double>(kd[c][2 * a], nb[c][2 * a], self[c]), ih2, lap);
        // D v: face +e_c (zero beyond a wall, wrapped when periodic) minus face c of this cell
        const double hi = pick<double>(kd[c][2 * c + 1], nb[c][2 * c + 1], self[c]);
        div = fmad(hi - (pin[c] ? 0.0 : self[c]), ih, div);
        out[c] = pin[c] ? 0.0 : fmad(-R.eta, lap, (pc - pm[c]) * ih);
    }
    out[3] = -div;
}

// Two consecutive values of x as FP64 (one load of two).
__device__ __forceinline__ void ld_pair(const double *q, double &a, double &b) {
    const double2 v = *reinterpret_cast<const double2 *>(q);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void ld_pair(const float *q, double &a, double &b) {
    const float2 v = *reinterpret_cast<const float2 *>(q);
    a = (double)v.x;
    b = (double)v.y;
}

// Two consecutive x cells per thread (rows of even length, blocks of 512 cells,
// fields aligned to two values): the pair, its y and z neighbour pairs and the
// pressure pairs move as one load each (x in FP64 or FP32, the preconditioned
// vectors of an FP32 preconditioner), the x neighbours outside the pair as scalars;
// the y and z rules are shared by the pair.  The output is FP64, 16-byte stores.
//
// Every gather is issued unconditionally (a neighbour a boundary rule ignores is
// read at a safe offset, the cell itself), and the raw values pass through an empty
// asm statement before the rules select among them.  Without that the compiler
// moves each load whose value some rule discards into a branch, where it waits for
// its data alone: the thread's twenty-odd gathers then run one after another.
template <typename TX>
__device__ __forceinline__ void ld_raw2(const TX *q, TX &a, TX &b);
template <>
__device__ __forceinline__ void ld_raw2<double>(const double *q, double &a, double &b) {
    const double2 v = *reinterpret_cast<const double2 *>(q);
    a = v.x;
    b = v.y;
}
template <>
__device__ __forceinline__ void ld_raw2<float>(const float *q, float &a, float &b) {
    const float2 v = *reinterpret_cast<const float2 *>(q);
    a = v.x;
    b = v.y;
}

// An offset the compiler cannot see through: a neighbour a rule ignores is read at
// offset 0 (the cell itself), and a visible 0 lets the compiler reuse the cell's own
// load under a branch instead of issuing the gather.
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

template <typename TX>
__device__ __forceinline__ void keep12(TX r[12]) {
    asm volatile("" : "+v"(r[0]), "+v"(r[1]), "+v"(r[2]), "+v"(r[3]), "+v"(r[4]), "+v"(r[5]), "+v"(r[6]),
                 "+v"(r[7]), "+v"(r[8]), "+v"(r[9]), "+v"(r[10]), "+v"(r[11]));
}

template <typename TX>
__device__ __forceinline__ void apply_row2(const RepDev &R, const BlockEnt &be, const TX *__restrict__ xr,
                                           double *__restrict__ yr) {
    const long long g0 = be.start + 2LL * threadIdx.x;
    if (g0 >= R.N) return;
    // the grid's sizes and rules, read once (the rules below would otherwise read them
    // lazily, each under its own branch)
    int nn[3] = {R.n[0], R.n[1], R.n[2]}, bcc[3] = {R.bc[0], R.bc[1], R.bc[2]};
    asm volatile("" : "+v"(nn[0]), "+v"(nn[1]), "+v"(nn[2]), "+v"(bcc[0]), "+v"(bcc[1]), "+v"(bcc[2]));
    const int lin = (int)g0, N = (int)R.N, n0 = nn[0];
    int idx[3];
    unlin(lin, R, idx);
    const int st[3] = {1, nn[0], nn[0] * nn[1]};
    const TX *p = xr + 3LL * N;
    int kd[2][3][6];
    // raw[c]: self pair, -y pair, +y pair, -z pair, +z pair, -x and +x beyond the pair;
    // raw[3]: the pressure pair, its -x value, -y pair, -z pair (one slot unused)
    TX raw[4][12];
    const int xm = idx[0] == 0 ? n0 - 1 : -1;                        // -x of the first cell
    const int xp = 1 + (idx[0] + 1 == n0 - 1 ? -(n0 - 1) : 1);      // +x of the second cell
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const TX *u = xr + (long long)c * N;
        ld_raw2<TX>(u + lin, raw[c][0], raw[c][1]);
#pragma unroll
        for (int a = 1; a < 3; ++a) {
            const int km = nbr_kind(idx[a], -1, nn[a], bcc[a], a, c);
            const int kp = nbr_kind(idx[a], +1, nn[a], bcc[a], a, c);
            const int om = opaque(km ? 0 : (idx[a] == 0 ? (nn[a] - 1) * st[a] : -st[a]));
            const int op = opaque(kp ? 0 : (idx[a] == nn[a] - 1 ? -(nn[a] - 1) * st[a] : st[a]));
            ld_raw2<TX>(u + lin + om, raw[c][4 * a - 2], raw[c][4 * a - 1]);
            ld_raw2<TX>(u + lin + op, raw[c][4 * a], raw[c][4 * a + 1]);
            kd[0][c][2 * a] = kd[1][c][2 * a] = km;
            kd[0][c][2 * a + 1] = kd[1][c][2 * a + 1] = kp;
        }
        raw[c][10] = u[lin + xm];
        raw[c][11] = u[lin + xp];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            kd[q][c][0] = nbr_kind(idx[0] + q, -1, n0, bcc[0], 0, c);
            kd[q][c][1] = nbr_kind(idx[0] + q, +1, n0, bcc[0], 0, c);
        }
    }
    ld_raw2<TX>(p + lin, raw[3][0], raw[3][1]);
    raw[3][2] = p[lin + (idx[0] > 0 ? -1 : n0 - 1)];
    ld_raw2<TX>(p + lin + (idx[1] > 0 ? -st[1] : (nn[1] - 1) * st[1]), raw[3][3], raw[3][4]);
    ld_raw2<TX>(p + lin + (idx[2] > 0 ? -st[2] : (nn[2] - 1) * st[2]), raw[3][5], raw[3][6]);
    raw[3][7] = raw[3][8] = raw[3][9] = raw[3][10] = raw[3][11] = (TX)0;
#pragma unroll
    for (int g = 0; g < 4; ++g) keep12<TX>(raw[g]);
    double self[2][3], nb[2][3][6], pm[2][3];
    bool pin[2][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double spx = (double)raw[c][0], spy = (double)raw[c][1];
        self[0][c] = spx;
        self[1][c] = spy;
#pragma unroll
        for (int a = 1; a < 3; ++a) {
            nb[0][c][2 * a] = (double)raw[c][4 * a - 2];
            nb[1][c][2 * a] = (double)raw[c][4 * a - 1];
            nb[0][c][2 * a + 1] = (double)raw[c][4 * a];
            nb[1][c][2 * a + 1] = (double)raw[c][4 * a + 1];
        }
        // x neighbours: inside the pair, or one cell beyond it (wrapped when periodic)
        nb[0][c][0] = kd[0][c][0] ? spx : (double)raw[c][10];
        nb[0][c][1] = spy;
        nb[1][c][0] = spx;
        nb[1][c][1] = kd[1][c][1] ? spy : (double)raw[c][11];
        pin[0][c] = bcc[c] != RBFIB_PERIODIC && (c == 0 ? idx[0] : idx[c]) == 0;
        pin[1][c] = bcc[c] != RBFIB_PERIODIC && (c == 0 ? idx[0] + 1 : idx[c]) == 0;
    }
    // pressure at -e_c
    pm[0][0] = (double)raw[3][2];
    pm[1][0] = (double)raw[3][0];
    pm[0][1] = (double)raw[3][3];
    pm[1][1] = (double)raw[3][4];
    pm[0][2] = (double)raw[3][5];
    pm[1][2] = (double)raw[3][6];
    const double pc0 = (double)raw[3][0], pc1 = (double)raw[3][1];
    double o0[4], o1[4];
    apply_cell(R, self[0], nb[0], pm[0], pc0, kd[0], pin[0], o0);
    apply_cell(R, self[1], nb[1], pm[1], pc1, kd[1], pin[1], o1);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        *reinterpret_cast<double2 *>(yr + (long long)c * N + lin) = make_double2(o0[c], o1[c]);
}

// One thread per cell (npt cells, RB_BLOCK apart), or apply_row2 where it applies.
// Neighbour offsets and boundary rules are computed first and applied with selects,
// so the loads of all three components are in flight together; the divergence
// reuses each component's +e_c neighbour.
template <typename TX>
__global__ __launch_bounds__(RB_BLOCK) void k_apply_fluid(const RepDev *reps, const BlockEnt *tab,
                                                          const TX *__restrict__ x, double *__restrict__ y,
                                                          const int *__restrict__ mask) {
    const BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    const TX *xr = x + R.off;
    double *yr = y + R.off;
    // uniform per block: even rows, even field length, fields aligned to two values
    if (be.npt == 2 && R.n[0] % 2 == 0 && R.N % 2 == 0 &&
        ((reinterpret_cast<unsigned long long>(xr) & (2 * sizeof(TX) - 1)) == 0) &&
        ((reinterpret_cast<unsigned long long>(yr) & 15) == 0)) {
        apply_row2(R, be, xr, yr);
        return;
    }
    for (int t_ = 0; t_ < be.npt; ++t_) {
    const long long l = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    if (l >= R.N) break;
    const int lin = (int)l, N = (int)R.N;
    int idx[3];
    unlin(lin, R, idx);
    const int st[3] = {1, R.n[0], R.n[0] * R.n[1]};
    int kd[3][6], off[3][6], offp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            kd[c][2 * a] = nbr_kind(idx[a], -1, R.n[a], R.bc[a], a, c);
            kd[c][2 * a + 1] = nbr_kind(idx[a], +1, R.n[a], R.bc[a], a, c);
            off[c][2 * a] = kd[c][2 * a] ? 0 : (idx[a] == 0 ? (R.n[a] - 1) * st[a] : -st[a]);
            off[c][2 * a + 1] = kd[c][2 * a + 1] ? 0 : (idx[a] == R.n[a] - 1 ? -(R.n[a] - 1) * st[a] : st[a]);
        }
        offp[c] = idx[c] > 0 ? -st[c] : (R.n[c] - 1) * st[c];   // pressure at -e_c (unused when pinned)
    }
    double self[3], nb[3][6], pm[3];
    bool pin[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const TX *u = xr + (long long)c * N;
        self[c] = (double)u[lin];
#pragma unroll
        for (int q = 0; q < 6; ++q) nb[c][q] = (double)u[lin + off[c][q]];
        pm[c] = (double)xr[3LL * N + lin + offp[c]];
        pin[c] = pinned(c, idx, R.bc);
    }
    double out[4];
    apply_cell(R, self, nb, pm, (double)xr[3LL * N + lin], kd, pin, out);
#pragma unroll
    for (int c = 0; c < 4; ++c) yr[(long long)c * N + lin] = out[c];
    }
}

// The same apply by z-marching: a workgroup owns an RB_AZT x RB_AZT tile of x-y
// cells and be.npt consecutive planes along z (be.start: linear index of the tile's
// first cell).  Each thread keeps its cell's four fields at planes k-1, k and k+1 in
// registers (plane k+2 is loaded one step ahead) and publishes plane k in LDS, where
// the tile's x and y neighbours are read; neighbours outside the tile (tile edges,
// periodic wraps) come from global memory.  A neighbour across a wall is never read
// (its rule ignores the value).  The gathered values are those of k_apply_fluid, so
// the results are identical.
// Neighbour of cell (i, j) along a = 0 (x) or 1 (y) in direction d, wrapped on a
// periodic axis: its slot in the tile (>= 0), or -1 with g its x-y offset in the
// plane when it lies outside the tile, or -2 beyond a wall.
__device__ __forceinline__ int az_nbr(int i, int j, int a, int d, int nx, int ny, int bca, int x0, int y0,
                                      long long &g) {
    int q0 = i, q1 = j;
    const int n = a == 0 ? nx : ny;
    int q = (a == 0 ? q0 : q1) + d;
    if (q < 0 || q >= n) {
        if (bca != RBFIB_PERIODIC) return -2;
        q += q < 0 ? n : -n;
    }
    if (a == 0) q0 = q; else q1 = q;
    const int lx = q0 - x0, ly = q1 - y0;
    if (lx >= 0 && lx < RB_AZT && ly >= 0 && ly < RB_AZT) return lx + RB_AZT * ly;
    g = q0 + (long long)nx * q1;
    return -1;
}

template <typename TX>
__device__ __forceinline__ void az_plane(const TX *__restrict__ xr, long long N, long long sxy, long long col, int k,
                                         int nz, bool zper, bool live, double v[4]) {
    const int kk = (k >= 0 && k < nz) ? k : (zper ? (k < 0 ? k + nz : k - nz) : -1);
#pragma unroll
    for (int f = 0; f < 4; ++f) v[f] = (live && kk >= 0) ? (double)xr[(long long)f * N + kk * sxy + col] : 0.0;
}

template <typename TX>
__global__ __launch_bounds__(RB_AZT *RB_AZT) void k_apply_fluid_z(const RepDev *reps, const BlockEnt *tab,
                                                                  const TX *__restrict__ x, double *__restrict__ y,
                                                                  const int *__restrict__ mask) {
    const BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    __shared__ double sh[2][4][RB_AZT * RB_AZT];
    const int nx = R.n[0], ny = R.n[1], nz = R.n[2];
    const long long N = R.N, sxy = (long long)nx * ny;
    int o[3];
    unlin(be.start, R, o);
    const int tx = threadIdx.x % RB_AZT, ty = threadIdx.x / RB_AZT;
    const int i = o[0] + tx, j = o[1] + ty;
    const bool live = i < nx && j < ny;
    const int z1 = min(o[2] + be.npt, nz);
    const TX *xr = x + R.off;
    double *yr = y + R.off;
    const long long col = live ? (long long)i + (long long)nx * j : 0;
    const bool zper = R.bc[2] == RBFIB_PERIODIC;
    // x and y neighbours of the thread's cell: slots or global offsets (fixed along z)
    long long gx[4] = {0, 0, 0, 0};
    int sl[4];
    sl[0] = az_nbr(i, j, 0, -1, nx, ny, R.bc[0], o[0], o[1], gx[0]);
    sl[1] = az_nbr(i, j, 0, +1, nx, ny, R.bc[0], o[0], o[1], gx[1]);
    sl[2] = az_nbr(i, j, 1, -1, nx, ny, R.bc[1], o[0], o[1], gx[2]);
    sl[3] = az_nbr(i, j, 1, +1, nx, ny, R.bc[1], o[0], o[1], gx[3]);
    double vm[4], v0[4], vp[4];
    az_plane(xr, N, sxy, col, o[2] - 1, nz, zper, live, vm);
    az_plane(xr, N, sxy, col, o[2], nz, zper, live, v0);
    az_plane(xr, N, sxy, col, o[2] + 1, nz, zper, live, vp);
    int b = 0;
    for (int k = o[2]; k < z1; ++k) {
        double vn[4];
        az_plane(xr, N, sxy, col, k + 2, nz, zper, live, vn);
#pragma unroll
        for (int f = 0; f < 4; ++f) sh[b][f][threadIdx.x] = v0[f];
        __syncthreads();
        if (live) {
            const int idx[3] = {i, j, k};
            double self[3], nb[3][6], pm[3];
            int kd[3][6];
            bool pin[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    kd[c][2 * a] = nbr_kind(idx[a], -1, R.n[a], R.bc[a], a, c);
                    kd[c][2 * a + 1] = nbr_kind(idx[a], +1, R.n[a], R.bc[a], a, c);
                }
                self[c] = v0[c];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double v = 0.0;
                    if (kd[c][q] == 0)
                        v = sl[q] >= 0 ? sh[b][c][sl[q]]
                                       : (sl[q] == -1 ? (double)xr[(long long)c * N + k * sxy + gx[q]] : 0.0);
                    nb[c][q] = v;
                }
                nb[c][4] = vm[c];
                nb[c][5] = vp[c];
                pin[c] = pinned(c, idx, R.bc);
            }
            // pressure at -e_c (unused where the face is pinned)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int q = 2 * c;
                double v = 0.0;
                if (!pin[c]) v = sl[q] >= 0 ? sh[b][3][sl[q]] : (sl[q] == -1 ? (double)xr[3 * N + k * sxy + gx[q]] : 0.0);
                pm[c] = v;
            }
            pm[2] = vm[3];
            double out[4];
            apply_cell(R, self, nb, pm, v0[3], kd, pin, out);
#pragma unroll
            for (int c = 0; c < 4; ++c) yr[(long long)c * N + k * sxy + col] = out[c];
        }
        b ^= 1;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            vm[f] = v0[f];
            v0[f] = vp[f];
            vp[f] = vn[f];
        }
    }
}

template <typename TX>
void launch_apply_fluid(Ctx &c, const TX *x, double *y) {
    if (c.n_tab_az > 0) {
        hipLaunchKernelGGL(k_apply_fluid_z<TX>, dim3(c.n_tab_az), dim3(RB_AZT * RB_AZT), 0, c.stream, c.d_reps,
                           c.d_tab_az, x, y, c.mask);
        return;
    }
    hipLaunchKernelGGL(k_apply_fluid<TX>, dim3(c.n_tab_cells2), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_tab_cells2, x, y, c.mask);
}
template void launch_apply_fluid<double>(Ctx &, const double *, double *);
template void launch_apply_fluid<float>(Ctx &, const float *, double *);

// ------------------------------------------------------------------ multigrid
// Level pools hold 4 fields per (replica, level): comp c at lev.off + c * lev.N.
// FP32 cell kernels on four consecutive x cells per thread: blocks of 1024 cells
// (four per thread), rows a multiple of four long, and the replica's FP64 state
// 16-byte aligned (the level pools always are for such rows).  Uniform per block.
template <typename P>
__device__ __forceinline__ bool cells_row4(const BlockEnt &be, const RepDev &R, const P *state) {
    return be.npt == 4 && R.n[0] % 4 == 0 && ((reinterpret_cast<unsigned long long>(state + R.off) & 15) == 0);
}

__device__ __forceinline__ double2 ld_d2(const double *q) { return *reinterpret_cast<const double2 *>(q); }
// four consecutive z values (16-byte aligned): FP64 as two 16-byte stores, FP32 as one
__device__ __forceinline__ void st_four(double *q, const double o[4]) {
    *reinterpret_cast<double2 *>(q) = make_double2(o[0], o[1]);
    *reinterpret_cast<double2 *>(q + 2) = make_double2(o[2], o[3]);
}
__device__ __forceinline__ void st_four(float *q, const double o[4]) {
    *reinterpret_cast<float4 *>(q) = make_float4((float)o[0], (float)o[1], (float)o[2], (float)o[3]);
}
__device__ __forceinline__ float4 ld_f4(const float *q) { return *reinterpret_cast<const float4 *>(q); }

// b (level 0) = src * f, f = rs[rep * rstride] (1 without rs)
template <typename T>
__global__ void k_to_level0(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                            const double *__restrict__ src, T *__restrict__ b, int c0, const int *__restrict__ mask,
                            const double *__restrict__ rs, int rstride) {
    BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &Lv = levs[be.rep * RB_MAXLEV];
    const double f = rs ? rs[(long long)be.rep * rstride] : 1.0;
    if constexpr (sizeof(T) == 4) {
        if (cells_row4(be, R, src)) {
            const long long lin = be.start + 4LL * threadIdx.x;
            if (lin >= R.N) return;
            const double *s = src + R.off + comp * R.N + lin;
            const double2 a = ld_d2(s), c = ld_d2(s + 2);
            *reinterpret_cast<float4 *>(b + Lv.off + comp * Lv.N + lin) =
                make_float4((float)(a.x * f), (float)(a.y * f), (float)(c.x * f), (float)(c.y * f));
            return;
        }
    }
    for (int t_ = 0; t_ < be.npt; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    if (lin >= R.N) continue;
    b[Lv.off + comp * Lv.N + lin] = (T)(src[R.off + comp * R.N + lin] * f);
    }
}

template <typename T>
void launch_to_level0(Ctx &c, const double *src, T *b, int c0, int nc, const double *rs) {
    hipLaunchKernelGGL(k_to_level0<T>, dim3(c.n_tab_cells, nc), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_levs,
                       c.d_tab_cells, src, b, c0, c.mask, rs, c.m + 1);
}

// Operator of component comp at a level: A = -eta Lm (velocity) or -L (pressure).
// MG_FIRST: damped Jacobi sweep from zero, x_out = w b (w = omega / diag);
// MG_SWEEP: x_out = x_in + w (b - A x_in); MG_RESID: x_out = b - A x_in.
// Pinned slots are written as zero.
// NPT points per thread, all loads of a thread issued before any arithmetic and
// the boundary rules applied with selects, so that the loads of the NPT points are
// in flight together.
// FP32 sweep on four consecutive x points per thread (rows whose length is a multiple
// of 4, blocks of 1024 points): 16-byte loads of the point, its y and z neighbour rows
// and b, two scalar loads for the x neighbours outside the group; y and z rules are
// shared by the four points.  Same arithmetic, in the same order, as the scalar path.
// MG_FIRST2 (four-point path only): the first two sweeps of a down pass in one.  The
// first sweep from zero leaves w1 b at every point it does not pin, so the second
// sweep rebuilds each value it reads from b (the neighbours it reads are never pinned
// ones) and x1 is never stored: b is read and x written once instead of 2 + 3 passes,
// with the values of the two separate sweeps.
#define MG_FIRST 0
#define MG_SWEEP 1
#define MG_RESID 2
#define MG_FIRST2 3

template <int MODE>
__device__ __forceinline__ void smooth_row4(const RepDev &R, const LevDev &Lv, const BlockEnt &be, int comp,
                                            const float *__restrict__ xi, float *__restrict__ xo,
                                            const float *__restrict__ bb, float s, float om, float om1) {
    const long long g0 = be.start + 4LL * threadIdx.x;
    if (g0 >= Lv.N) return;
    const int lin = (int)g0;
    int idx[3];
    unlin(lin, Lv, idx);
    const int n0 = Lv.n[0], x0 = idx[0];
    const int st[3] = {1, n0, n0 * Lv.n[1]};
    int kyz[4], off[4];
#pragma unroll
    for (int a = 1; a < 3; ++a) {
        const int km = nbr_kind(idx[a], -1, Lv.n[a], R.bc[a], a, comp);
        const int kp = nbr_kind(idx[a], +1, Lv.n[a], R.bc[a], a, comp);
        kyz[2 * (a - 1)] = km;
        kyz[2 * (a - 1) + 1] = kp;
        off[2 * (a - 1)] = km ? 0 : (idx[a] == 0 ? (Lv.n[a] - 1) * st[a] : -st[a]);
        off[2 * (a - 1) + 1] = kp ? 0 : (idx[a] == Lv.n[a] - 1 ? -(Lv.n[a] - 1) * st[a] : st[a]);
    }
    const float4 bv = *reinterpret_cast<const float4 *>(bb + lin);
    const float b4[4] = {bv.x, bv.y, bv.z, bv.w};
    float x4[4] = {0.f, 0.f, 0.f, 0.f}, nb[4][4], xl = 0.f, xr = 0.f;
    int kxm[4], kxp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        kxm[q] = nbr_kind(x0 + q, -1, n0, R.bc[0], 0, comp);
        kxp[q] = nbr_kind(x0 + q, +1, n0, R.bc[0], 0, comp);
    }
    // MG_FIRST2 reads these from b and scales them below
    const float *xs = MODE == MG_FIRST2 ? bb : xi;
    if (MODE != MG_FIRST) {
        const float4 v = *reinterpret_cast<const float4 *>(xs + lin);
        x4[0] = v.x; x4[1] = v.y; x4[2] = v.z; x4[3] = v.w;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float4 u = *reinterpret_cast<const float4 *>(xs + lin + off[e]);
            nb[e][0] = u.x; nb[e][1] = u.y; nb[e][2] = u.z; nb[e][3] = u.w;
        }
        // x neighbours outside the group (wrapped when periodic, unused otherwise)
        xl = xs[lin + (kxm[0] ? 0 : (x0 == 0 ? n0 - 1 : -1))];
        xr = xs[lin + 3 + (kxp[3] ? 0 : (x0 + 3 == n0 - 1 ? -(n0 - 1) : 1))];
    }
    const float ihx = (float)Lv.inv_h2[0], ihy = (float)Lv.inv_h2[1], ihz = (float)Lv.inv_h2[2];
    const float day = diag_axis<float>(comp, 1, idx[1], Lv.n[1], R.bc[1]);
    const float daz = diag_axis<float>(comp, 2, idx[2], Lv.n[2], R.bc[2]);
    // The diagonal's x term is the interior one except at x = 0 and x = n0 - 1 of a
    // tangential component on an x wall, which only the group's first and last points
    // can be (rows are a multiple of 4 long), so each weight is formed once per distinct
    // diagonal: interior, and at the row ends of the threads that hold them.
    const bool e0 = R.bc[0] != RBFIB_PERIODIC && comp != 0 && x0 == 0;
    const bool e3 = R.bc[0] != RBFIB_PERIODIC && comp != 0 && x0 + 3 == n0 - 1;
    const float xti = fmad(diag_axis<float>(comp, 0, x0 + 1, n0, R.bc[0]), ihx, 0.f);
    const float xte = fmad(diag_axis<float>(comp, 0, 0, n0, R.bc[0]), ihx, 0.f);
    const float wi = jacobi_w<float>(om, s, fmad(daz, ihz, fmad(day, ihy, xti)));
    float we = wi;
    if (e0 || e3) we = jacobi_w<float>(om, s, fmad(daz, ihz, fmad(day, ihy, xte)));
    if (MODE == MG_FIRST2) {
        // x1 = w1 b, with w1 from the diagonal of the point read.  The points outside the
        // group are interior or periodic, whose x term is the interior one; the y and z
        // neighbours differ from the point in one term, and only next to a y or z wall.
        const float dym = diag_axis<float>(comp, 1, idx[1] - 1, Lv.n[1], R.bc[1]);
        const float dyp = diag_axis<float>(comp, 1, idx[1] + 1, Lv.n[1], R.bc[1]);
        const float dzm = diag_axis<float>(comp, 2, idx[2] - 1, Lv.n[2], R.bc[2]);
        const float dzp = diag_axis<float>(comp, 2, idx[2] + 1, Lv.n[2], R.bc[2]);
        // weights of the point and of its four y / z neighbours, interior x term (v) and
        // wall x term (u)
        float v[5], u[5];
        v[0] = jacobi_w<float>(om1, s, fmad(daz, ihz, fmad(day, ihy, xti)));
        u[0] = v[0];
        if (e0 || e3) u[0] = jacobi_w<float>(om1, s, fmad(daz, ihz, fmad(day, ihy, xte)));
#pragma unroll
        for (int k = 1; k < 5; ++k) { v[k] = v[0]; u[k] = u[0]; }
        if (dym != day || dyp != day || dzm != daz || dzp != daz) {
            auto w4 = [&](float xt, float w[5]) {
                w[1] = jacobi_w<float>(om1, s, fmad(daz, ihz, fmad(dym, ihy, xt)));
                w[2] = jacobi_w<float>(om1, s, fmad(daz, ihz, fmad(dyp, ihy, xt)));
                w[3] = jacobi_w<float>(om1, s, fmad(dzm, ihz, fmad(day, ihy, xt)));
                w[4] = jacobi_w<float>(om1, s, fmad(dzp, ihz, fmad(day, ihy, xt)));
            };
            w4(xti, v);
            if (e0 || e3) w4(xte, u);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool eq = (q == 0 && e0) || (q == 3 && e3);
            x4[q] = x4[q] * (eq ? u[0] : v[0]);
#pragma unroll
            for (int e = 0; e < 4; ++e) nb[e][q] = nb[e][q] * (eq ? u[e + 1] : v[e + 1]);
        }
        xl = xl * v[0];
        xr = xr * v[0];
    }
    const bool pin_yz = (comp == 1 && R.bc[1] != RBFIB_PERIODIC && idx[1] == 0) ||
                        (comp == 2 && R.bc[2] != RBFIB_PERIODIC && idx[2] == 0);
    float y4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float w = ((q == 0 && e0) || (q == 3 && e3)) ? we : wi;
        float y;
        if (MODE == MG_FIRST) {
            y = b4[q] * w;
        } else {
            const float self = x4[q];
            const float xm = q == 0 ? xl : x4[q > 0 ? q - 1 : 0];
            const float xp = q == 3 ? xr : x4[q < 3 ? q + 1 : 3];
            float acc = lap_acc<float>(pick<float>(kxp[q], xp, self), self, pick<float>(kxm[q], xm, self), ihx, 0.f);
            acc = lap_acc<float>(pick<float>(kyz[1], nb[1][q], self), self, pick<float>(kyz[0], nb[0][q], self), ihy,
                                 acc);
            acc = lap_acc<float>(pick<float>(kyz[3], nb[3][q], self), self, pick<float>(kyz[2], nb[2][q], self), ihz,
                                 acc);
            y = MODE == MG_RESID ? mg_residual<float>(b4[q], s, acc) : jacobi_step<float>(self, b4[q], s, acc, w);
        }
        const bool pin = pin_yz || (comp == 0 && R.bc[0] != RBFIB_PERIODIC && x0 + q == 0);
        y4[q] = pin ? 0.f : y;
    }
    *reinterpret_cast<float4 *>(xo + lin) = make_float4(y4[0], y4[1], y4[2], y4[3]);
}

// One-point MG_FIRST2 (any precision, any level): the first iterate at the point is
// b w1 and at each neighbour the second sweep reads (never a pinned one) b(q) w1(q),
// with q's own diagonal formed in the first sweep's order; every value equals the
// separate sweeps'.
template <typename T>
__device__ __forceinline__ T first2_point(const RepDev &R, const LevDev &Lv, int comp, int li, const int idx[3],
                                          const T *__restrict__ bb, T s, T om1, T om2) {
    const int st[3] = {1, Lv.n[0], Lv.n[0] * Lv.n[1]};
    T da[3];
    int km[3], kp[3], om[3], op[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        da[a] = diag_axis<T>(comp, a, idx[a], Lv.n[a], R.bc[a]);
        km[a] = nbr_kind(idx[a], -1, Lv.n[a], R.bc[a], a, comp);
        kp[a] = nbr_kind(idx[a], +1, Lv.n[a], R.bc[a], a, comp);
        om[a] = km[a] ? 0 : (idx[a] == 0 ? (Lv.n[a] - 1) * st[a] : -st[a]);
        op[a] = kp[a] ? 0 : (idx[a] == Lv.n[a] - 1 ? -(Lv.n[a] - 1) * st[a] : st[a]);
    }
    const T ih[3] = {(T)Lv.inv_h2[0], (T)Lv.inv_h2[1], (T)Lv.inv_h2[2]};
    const T d = fmad(da[2], ih[2], fmad(da[1], ih[1], fmad(da[0], ih[0], (T)0)));
    const T bp = bb[li];
    T bq[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bq[2 * a] = bb[li + om[a]];
        bq[2 * a + 1] = bb[li + op[a]];
    }
    const T x1p = bp * jacobi_w<T>(om1, s, d);
    T acc = (T)0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T nbv[2];
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
            const int kind = dir ? kp[a] : km[a];
            T x1q = x1p;
            if (kind == 0) {
                int qa = idx[a] + (dir ? 1 : -1);
                qa = qa < 0 ? qa + Lv.n[a] : (qa >= Lv.n[a] ? qa - Lv.n[a] : qa);
                T dd[3] = {da[0], da[1], da[2]};
                dd[a] = diag_axis<T>(comp, a, qa, Lv.n[a], R.bc[a]);
                const T dq = fmad(dd[2], ih[2], fmad(dd[1], ih[1], fmad(dd[0], ih[0], (T)0)));
                x1q = bq[2 * a + dir] * jacobi_w<T>(om1, s, dq);
            }
            nbv[dir] = x1q;
        }
        acc = lap_acc<T>(pick<T>(kp[a], nbv[1], x1p), x1p, pick<T>(km[a], nbv[0], x1p), ih[a], acc);
    }
    return jacobi_step<T>(x1p, bp, s, acc, jacobi_w<T>(om2, s, d));
}

template <typename T, int NPT, int MODE>
__global__ __launch_bounds__(RB_BLOCK) void k_smooth(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                     int lev, int c0, const T *__restrict__ xin, T *__restrict__ xout,
                                                     const T *__restrict__ b, double omega,
                                                     const int *__restrict__ mask, double omega1) {
    const BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &Lv = levs[be.rep * RB_MAXLEV + lev];
    const long long base = Lv.off + comp * Lv.N;
    const T *xi = xin + base;
    const T *bb = b + base;
    T *xo = xout + base;
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    if constexpr (sizeof(T) == 4 && NPT == 4) {
        if (Lv.n[0] % 4 == 0) {    // uniform per block: every row splits into aligned groups of 4
            smooth_row4<MODE>(R, Lv, be, comp, (const float *)xi, (float *)xo, (const float *)bb, (float)s,
                              (float)omega, (float)omega1);
            return;
        }
    }
    if constexpr (MODE == MG_FIRST2) {
#pragma unroll
        for (int t = 0; t < NPT; ++t) {
            const long long l = be.start + threadIdx.x + (long long)t * RB_BLOCK;
            if (l >= Lv.N) break;
            const int li = (int)l;
            int idx[3];
            unlin(li, Lv, idx);
            const T y = first2_point<T>(R, Lv, comp, li, idx, bb, s, (T)omega1, (T)omega);
            xo[li] = pinned(comp, idx, R.bc) ? (T)0 : y;
        }
        return;
    }
    const int st[3] = {1, Lv.n[0], Lv.n[0] * Lv.n[1]};
    int lin[NPT], kinds[NPT];
    bool ok[NPT], pin[NPT];
    T dg[NPT], bv[NPT], xv[NPT], nb[NPT][6];
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
        const long long l = be.start + threadIdx.x + (long long)t * RB_BLOCK;
        ok[t] = l < Lv.N;
        lin[t] = ok[t] ? (int)l : 0;
        int idx[3];
        unlin(lin[t], Lv, idx);
        pin[t] = pinned(comp, idx, R.bc);
        T d = (T)0;
        int kd = 0;
        int off[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d = fmad(diag_axis<T>(comp, a, idx[a], Lv.n[a], R.bc[a]), (T)Lv.inv_h2[a], d);
            const int km = nbr_kind(idx[a], -1, Lv.n[a], R.bc[a], a, comp);
            const int kp = nbr_kind(idx[a], +1, Lv.n[a], R.bc[a], a, comp);
            kd |= (km | (kp << 2)) << (4 * a);
            // periodic neighbours wrap; the other rules never read the neighbour
            off[2 * a] = km ? 0 : (idx[a] == 0 ? (Lv.n[a] - 1) * st[a] : -st[a]);
            off[2 * a + 1] = kp ? 0 : (idx[a] == Lv.n[a] - 1 ? -(Lv.n[a] - 1) * st[a] : st[a]);
        }
        dg[t] = d;
        kinds[t] = kd;
        bv[t] = bb[lin[t]];
        if (MODE != MG_FIRST) {
            xv[t] = xi[lin[t]];
#pragma unroll
            for (int q = 0; q < 6; ++q) nb[t][q] = xi[lin[t] + off[q]];
        }
    }
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
        const T w = jacobi_w<T>((T)omega, s, dg[t]);
        T y;
        if (MODE == MG_FIRST) {
            y = bv[t] * w;
        } else {
            T acc = (T)0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int kd = kinds[t] >> (4 * a);
                acc = lap_acc<T>(pick<T>((kd >> 2) & 3, nb[t][2 * a + 1], xv[t]), xv[t],
                                 pick<T>(kd & 3, nb[t][2 * a], xv[t]), (T)Lv.inv_h2[a], acc);
            }
            y = MODE == MG_RESID ? mg_residual<T>(bv[t], s, acc) : jacobi_step<T>(xv[t], bv[t], s, acc, w);
        }
        if (ok[t]) xo[lin[t]] = pin[t] ? (T)0 : y;
    }
}

// The four-point path alone, for levels whose rows are all a multiple of four long:
// without the one-point fallback in the same kernel it needs far fewer registers, so
// more waves are resident to cover the stencil's load latency.
template <int MODE>
__global__ __launch_bounds__(RB_BLOCK) void k_smooth_row4(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                          int lev, int c0, const float *__restrict__ xin,
                                                          float *__restrict__ xout, const float *__restrict__ b,
                                                          double omega, const int *__restrict__ mask,
                                                          double omega1) {
    const BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &Lv = levs[be.rep * RB_MAXLEV + lev];
    const long long base = Lv.off + comp * Lv.N;
    const float s = (comp < 3) ? (float)(-R.eta) : -1.f;
    smooth_row4<MODE>(R, Lv, be, comp, xin + base, xout + base, b + base, s, (float)omega, (float)omega1);
}

// omega1: the first sweep's weight of MG_FIRST2 (ignored by the other modes)
template <typename T, int NPT, int MODE>
static void launch_stencil(Ctx &c, int lev, int c0, int nc, const T *xin, T *xout, const T *b, double omega,
                           double omega1) {
    if constexpr (sizeof(T) == 4 && NPT == 4) {
        if (c.lev_row4[lev]) {
            hipLaunchKernelGGL(k_smooth_row4<MODE>, dim3(c.n_tab_lev[lev], nc), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                               c.d_levs, c.d_tab_lev[lev], lev, c0, (const float *)xin, (float *)xout,
                               (const float *)b, omega, c.mask, omega1);
            return;
        }
    }
    hipLaunchKernelGGL((k_smooth<T, NPT, MODE>), dim3(c.n_tab_lev[lev], nc), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_levs, c.d_tab_lev[lev], lev, c0, xin, xout, b, omega, c.mask, omega1);
}

template <typename T, int MODE>
static void launch_stencil_any(Ctx &c, int lev, int c0, int nc, const T *xin, T *xout, const T *b, double omega,
                               double omega1 = 0.0) {
    if (c.n_tab_lev[lev] == 0) return;
    if (MODE != MG_FIRST2) omega1 = omega;
    if (c.mg_npt == 4) launch_stencil<T, 4, MODE>(c, lev, c0, nc, xin, xout, b, omega, omega1);
    else launch_stencil<T, 1, MODE>(c, lev, c0, nc, xin, xout, b, omega, omega1);
}

// one damped-Jacobi sweep with weight omega (first: from a zero iterate)
template <typename T>
void launch_smooth(Ctx &c, int lev, int c0, int nc, const T *xin, T *xout, const T *b, bool first, double omega) {
    if (first) launch_stencil_any<T, MG_FIRST>(c, lev, c0, nc, xin, xout, b, omega);
    else launch_stencil_any<T, MG_SWEEP>(c, lev, c0, nc, xin, xout, b, omega);
}

// The first two sweeps of a down pass (weights omega1, omega2) as one launch: the
// four-point kernel on FP32 levels whose rows are a multiple of 4, the one-point
// kernel elsewhere (either precision).  Returns true (something launched or nothing
// to do).
template <typename T>
bool launch_smooth_first2(Ctx &c, int lev, int c0, int nc, T *xout, const T *b, double omega1, double omega2) {
    launch_stencil_any<T, MG_FIRST2>(c, lev, c0, nc, b, xout, b, omega2, omega1);
    return true;
}

// Restriction of the residual r of level lev (written by a MG_RESID pass, zero at
// pinned points) to the right-hand side of level lev+1: face-normal axis full
// weighting (1/4, 1/2, 1/4 on faces 2I-1, 2I, 2I+1), cell-centred axes averaging of
// the two children; an axis that is not coarsened keeps its index.
template <typename T, int NPT>
__global__ __launch_bounds__(RB_BLOCK) void k_restrict(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                       int lev, int c0, const T *__restrict__ rpool,
                                                       T *__restrict__ bcpool, const int *__restrict__ mask) {
    BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    const T *rf = rpool + F.off + comp * F.N;
    bool crs[3], face[3];
    int fc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        crs[a] = F.n[a] != C.n[a];
        face[a] = crs[a] && a == comp;
        fc[a] = !crs[a] ? 1 : (face[a] ? 3 : 2);
    }
    const int f01 = F.n[0] * F.n[1];
    // periodic wrap of the face-normal neighbours (wall: ci = 0 is pinned, excluded below)
    auto wrap = [](int f, int n) { return f < 0 ? f + n : (f >= n ? f - n : f); };
#pragma unroll
    for (int t_ = 0; t_ < NPT; ++t_) {
        long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
        if (lin >= C.N) continue;
        int ci[3];
        unlin(lin, C, ci);
        long long cbase = C.off + comp * C.N;
        if (pinned(comp, ci, R.bc)) { bcpool[cbase + lin] = (T)0; continue; }
        int fb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) fb[a] = crs[a] ? 2 * ci[a] - (face[a] ? 1 : 0) : ci[a];
        T acc = (T)0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                for (int ii = 0; ii < 3; ++ii)
                    if (kk < fc[2] && jj < fc[1] && ii < fc[0])
                        acc = fmad(restrict_weight<T>(crs[0], face[0], ii) * restrict_weight<T>(crs[1], face[1], jj) *
                                       restrict_weight<T>(crs[2], face[2], kk),
                                   rf[wrap(fb[0] + ii, F.n[0]) + F.n[0] * wrap(fb[1] + jj, F.n[1]) +
                                      f01 * wrap(fb[2] + kk, F.n[2])],
                                   acc);
        bcpool[cbase + lin] = acc;
    }
}

// B(lev+1) = R (B(lev) - A X(lev)); the residual passes through r (same pool layout).
template <typename T>
void launch_restrict(Ctx &c, int lev, int c0, int nc, const T *x, const T *b, T *bcoarse, T *r) {
    if (c.n_tab_lev[lev] == 0) return;
    launch_stencil_any<T, MG_RESID>(c, lev, c0, nc, x, r, b, c.opts.mg_omega);   // the residual ignores omega
    // one thread per coarse point: the table of level lev+1 restricted to replicas descending from lev
    if (c.mg_npt == 4)
        hipLaunchKernelGGL((k_restrict<T, 4>), dim3(c.n_tab_all[lev + 1], nc), dim3(RB_BLOCK), 0, c.stream,
                           c.d_reps, c.d_levs, c.d_tab_all[lev + 1], lev, c0, r, bcoarse, c.mask);
    else
        hipLaunchKernelGGL((k_restrict<T, 1>), dim3(c.n_tab_all[lev + 1], nc), dim3(RB_BLOCK), 0, c.stream,
                           c.d_reps, c.d_levs, c.d_tab_all[lev + 1], lev, c0, r, bcoarse, c.mask);
}

// x_f += P x_c: face-normal axis linear (even faces copy, odd faces average),
// cell-centred axes linear (3/4, 1/4) with odd ghosts for velocity at walls and
// even ghosts for pressure.
//
// FP32 path on four consecutive fine x points (rows a multiple of four long, blocks
// of 1024 points): x_f moves as one float4; the y/z weights are shared; per coarse
// (y, z) row the four coarse x values the group can use (indices base .. base+3,
// wrapped or clamped like prolong_axis) are loaded once and picked by index.  The
// sums run in prolong_at's order, so the values are identical.
__device__ __forceinline__ void prolong_row4(const RepDev &R, const LevDev &F, const LevDev &C, const BlockEnt &be,
                                             int comp, const float *__restrict__ xc, float *__restrict__ xf) {
    const long long g0 = be.start + 4LL * threadIdx.x;
    if (g0 >= F.N) return;
    const int lin = (int)g0;
    int fi[3];
    unlin(lin, F, fi);
    const int x0 = fi[0];
    const bool crsx = F.n[0] != C.n[0];
    const int base = crsx ? (x0 >> 1) - 1 : x0;
    int cx[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int i = base + t;
        if (R.bc[0] == RBFIB_PERIODIC) i = i < 0 ? i + C.n[0] : (i >= C.n[0] ? i - C.n[0] : i);
        else i = i < 0 ? 0 : (i >= C.n[0] ? C.n[0] - 1 : i);
        cx[t] = i;
    }
    const ProlongAxis<float> py = prolong_axis<float>(fi[1], F.n[1], C.n[1], R.bc[1], comp == 1, comp);
    const ProlongAxis<float> pz = prolong_axis<float>(fi[2], F.n[2], C.n[2], R.bc[2], comp == 2, comp);
    const long long c01 = (long long)C.n[0] * C.n[1];
    float rowv[2][2][4];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const bool use = kk < pz.cnt && jj < py.cnt;
            const long long ro = (long long)C.n[0] * (jj ? py.i1 : py.i0) + c01 * (kk ? pz.i1 : pz.i0);
#pragma unroll
            for (int t = 0; t < 4; ++t) rowv[kk][jj][t] = use ? xc[ro + cx[t]] : 0.f;
        }
    const float4 v = *reinterpret_cast<const float4 *>(xf + lin);
    float x4[4] = {v.x, v.y, v.z, v.w};
    const bool pin_yz = (comp == 1 && R.bc[1] != RBFIB_PERIODIC && fi[1] == 0) ||
                        (comp == 2 && R.bc[2] != RBFIB_PERIODIC && fi[2] == 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (pin_yz || (comp == 0 && R.bc[0] != RBFIB_PERIODIC && x0 + q == 0)) continue;
        const ProlongAxis<float> px = prolong_axis<float>(x0 + q, F.n[0], C.n[0], R.bc[0], comp == 0, comp);
        float acc = 0.f;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                for (int ii = 0; ii < 2; ++ii)
                    if (kk < pz.cnt && jj < py.cnt && ii < px.cnt) {
                        const int i = ii ? px.i1 : px.i0;
                        const float *rv = rowv[kk][jj];
                        const float cv = i == cx[0] ? rv[0] : (i == cx[1] ? rv[1] : (i == cx[2] ? rv[2] : rv[3]));
                        acc = fmad((ii ? px.w1 : px.w0) * (jj ? py.w1 : py.w0) * (kk ? pz.w1 : pz.w0), cv, acc);
                    }
        x4[q] += acc;
    }
    *reinterpret_cast<float4 *>(xf + lin) = make_float4(x4[0], x4[1], x4[2], x4[3]);
}

template <typename T, int NPT>
__global__ __launch_bounds__(RB_BLOCK) void k_prolong(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                      int lev, int c0, const T *__restrict__ xc, T *__restrict__ xf,
                                                      const int *__restrict__ mask) {
    BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    if constexpr (sizeof(T) == 4 && NPT == 4) {
        if (F.n[0] % 4 == 0) {    // uniform per block
            prolong_row4(R, F, C, be, comp, (const float *)(xc + C.off + comp * C.N), (float *)(xf + F.off + comp * F.N));
            return;
        }
    }
    for (int t_ = 0; t_ < NPT; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    if (lin >= F.N) continue;
    int fi[3];
    unlin(lin, F, fi);
    if (pinned(comp, fi, R.bc)) continue;
    const T acc = prolong_at<T>(R, F, C, comp, fi, xc + C.off + comp * C.N);
    xf[F.off + comp * F.N + lin] += acc;
    }
}

template <typename T>
void launch_prolong(Ctx &c, int lev, int c0, int nc, const T *xc, T *xf) {
    if (c.n_tab_lev[lev] == 0) return;
    if (c.mg_npt == 4)
        hipLaunchKernelGGL((k_prolong<T, 4>), dim3(c.n_tab_lev[lev], nc), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                           c.d_levs, c.d_tab_lev[lev], lev, c0, xc, xf, c.mask);
    else
        hipLaunchKernelGGL((k_prolong<T, 1>), dim3(c.n_tab_lev[lev], nc), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                           c.d_levs, c.d_tab_lev[lev], lev, c0, xc, xf, c.mask);
}

// Dense coarsest solve x = Ainv b, one workgroup per (replica, component).
template <typename T>
__global__ void k_coarse(const RepDev *reps, const LevDev *levs, const BlockEnt *tab, int lev, int c0,
                         const long long *coff, const T *__restrict__ Ainv, const T *__restrict__ b,
                         T *__restrict__ x, const int *__restrict__ mask) {
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    int comp = c0 + blockIdx.y;
    const LevDev &Lv = levs[be.rep * RB_MAXLEV + lev];
    extern __shared__ unsigned char smem_raw[];
    T *bs = reinterpret_cast<T *>(smem_raw);
    int m = (int)Lv.N;
    const T *bb = b + Lv.off + comp * Lv.N;
    for (int i = threadIdx.x; i < m; i += blockDim.x) bs[i] = bb[i];
    __syncthreads();
    const T *A = Ainv + coff[be.rep * 4 + comp];
    T *xx = x + Lv.off + comp * Lv.N;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        T acc = (T)0;
        const T *row = A + (long long)i * m;
        for (int j = 0; j < m; ++j) acc = fmad(row[j], bs[j], acc);
        xx[i] = acc;
    }
}

template <typename T> const T *coarse_pool(Ctx &c);
template <> const double *coarse_pool<double>(Ctx &c) { return c.d_coarse64; }
template <> const float *coarse_pool<float>(Ctx &c) { return c.d_coarse32; }

template <typename T>
void launch_coarse(Ctx &c, int lev, int c0, int nc, const T *b, T *x) {
    if (c.n_tab_crs[lev] == 0) return;
    size_t sh = sizeof(T) * (size_t)c.max_coarse;
    hipLaunchKernelGGL(k_coarse<T>, dim3(c.n_tab_crs[lev], nc), dim3(RB_BLOCK), sh, c.stream, c.d_reps, c.d_levs,
                       c.d_tab_crs[lev], lev, c0, c.d_coarse_off, coarse_pool<T>(c), b, x, c.mask);
}

// ------------------------------------------------------------------ bottom of the V-cycle in LDS
// One workgroup per (replica, component) runs the levels lb .. nlev-1 of its replica
// (lb = RepDev::lb, the first level whose grids fit MGB_LDS bytes) with every grid
// in LDS: the down sweeps, residual and restriction of each level, the dense
// coarsest solve, and the prolongation and up sweeps, separated by workgroup
// barriers instead of kernel launches.  Every point is computed by the helpers
// and in the operation order of the separate kernels, so the result is the same
// to the bit.  LDS: x_l and b_l for l = lb .. nlev-1, then one level-lb scratch
// grid t for the Jacobi ping-pong and the residual.
// Work split of a pass: a level of n01 (i, j) columns is cut into S slices per
// column (S = threads / columns on levels with fewer columns than threads, else 1),
// slice s taking the planes s, s + S, ...; the x and y boundary rules, the x and y
// terms of the diagonal and the pinning in x and y are evaluated once per column
// slice.  Input and output grids share one LDS array, so the compiler cannot move
// a load above an earlier store: a sweep therefore loads RB_BOTK planes of its
// slice (clamped to the last plane, never out of the grid) before it stores any,
// and the transfers load every point of their stencil before selecting the terms
// that count.
#define RB_BOTK 4

__device__ __forceinline__ int bot_slices(int ncol) {
    return ncol >= (int)blockDim.x ? 1 : (int)blockDim.x / ncol;
}

template <typename T, int MODE>
__device__ __forceinline__ void bot_sweep(const RepDev &R, const LevDev &Lv, int comp, T s, T om,
                                          const T *xi, T *xo, const T *bb) {
    const int n0 = Lv.n[0], n1 = Lv.n[1], n2 = Lv.n[2], n01 = n0 * n1;
    const T ih0 = (T)Lv.inv_h2[0], ih1 = (T)Lv.inv_h2[1], ih2 = (T)Lv.inv_h2[2];
    const int S = bot_slices(n01);
    for (int cs = threadIdx.x; cs < n01 * S; cs += blockDim.x) {
        const int sl = cs / n01, col = cs - sl * n01;
        const int j = col / n0, i = col - j * n0;
        const int kxm = nbr_kind(i, -1, n0, R.bc[0], 0, comp), kxp = nbr_kind(i, +1, n0, R.bc[0], 0, comp);
        const int kym = nbr_kind(j, -1, n1, R.bc[1], 1, comp), kyp = nbr_kind(j, +1, n1, R.bc[1], 1, comp);
        const int oxm = kxm ? 0 : (i == 0 ? n0 - 1 : -1);
        const int oxp = kxp ? 0 : (i == n0 - 1 ? -(n0 - 1) : 1);
        const int oym = kym ? 0 : (j == 0 ? (n1 - 1) * n0 : -n0);
        const int oyp = kyp ? 0 : (j == n1 - 1 ? -(n1 - 1) * n0 : n0);
        const T dxy = fmad(diag_axis<T>(comp, 1, j, n1, R.bc[1]), ih1,
                           fmad(diag_axis<T>(comp, 0, i, n0, R.bc[0]), ih0, (T)0));
        const bool pin_xy = (comp == 0 && R.bc[0] != RBFIB_PERIODIC && i == 0) ||
                            (comp == 1 && R.bc[1] != RBFIB_PERIODIC && j == 0);
        for (int k0 = sl; k0 < n2; k0 += RB_BOTK * S) {
            T bv[RB_BOTK], xv[RB_BOTK], vxp[RB_BOTK], vxm[RB_BOTK], vyp[RB_BOTK], vym[RB_BOTK], vzp[RB_BOTK],
                vzm[RB_BOTK];
            int kzm[RB_BOTK], kzp[RB_BOTK];
#pragma unroll
            for (int u = 0; u < RB_BOTK; ++u) {
                const int k = min(k0 + u * S, n2 - 1);
                const int lin = col + k * n01;
                bv[u] = bb[lin];
                if (MODE != MG_FIRST) {
                    kzm[u] = nbr_kind(k, -1, n2, R.bc[2], 2, comp);
                    kzp[u] = nbr_kind(k, +1, n2, R.bc[2], 2, comp);
                    const int ozm = kzm[u] ? 0 : (k == 0 ? (n2 - 1) * n01 : -n01);
                    const int ozp = kzp[u] ? 0 : (k == n2 - 1 ? -(n2 - 1) * n01 : n01);
                    xv[u] = xi[lin];
                    vxp[u] = xi[lin + oxp];
                    vxm[u] = xi[lin + oxm];
                    vyp[u] = xi[lin + oyp];
                    vym[u] = xi[lin + oym];
                    vzp[u] = xi[lin + ozp];
                    vzm[u] = xi[lin + ozm];
                }
            }
#pragma unroll
            for (int u = 0; u < RB_BOTK; ++u) {
                const int k = k0 + u * S;
                if (k < n2) {
                    const int lin = col + k * n01;
                    const T d = fmad(diag_axis<T>(comp, 2, k, n2, R.bc[2]), ih2, dxy);
                    const T w = jacobi_w<T>(om, s, d);
                    T y;
                    if (MODE == MG_FIRST) {
                        y = bv[u] * w;
                    } else {
                        T acc = lap_acc<T>(pick<T>(kxp, vxp[u], xv[u]), xv[u], pick<T>(kxm, vxm[u], xv[u]), ih0, (T)0);
                        acc = lap_acc<T>(pick<T>(kyp, vyp[u], xv[u]), xv[u], pick<T>(kym, vym[u], xv[u]), ih1, acc);
                        acc = lap_acc<T>(pick<T>(kzp[u], vzp[u], xv[u]), xv[u], pick<T>(kzm[u], vzm[u], xv[u]), ih2,
                                         acc);
                        y = MODE == MG_RESID ? mg_residual<T>(bv[u], s, acc) : jacobi_step<T>(xv[u], bv[u], s, acc, w);
                    }
                    const bool pin = pin_xy || (comp == 2 && R.bc[2] != RBFIB_PERIODIC && k == 0);
                    xo[lin] = pin ? (T)0 : y;
                }
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ void bot_restrict(const RepDev &R, const LevDev &F, const LevDev &C, int comp,
                                             const T *rf, T *bc) {
    bool crs[3], face[3];
    int fc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        crs[a] = F.n[a] != C.n[a];
        face[a] = crs[a] && a == comp;
        fc[a] = !crs[a] ? 1 : (face[a] ? 3 : 2);
    }
    const int f01 = F.n[0] * F.n[1], c01 = C.n[0] * C.n[1];
    auto wrap = [](int f, int n) { return f < 0 ? f + n : (f >= n ? f - n : f); };
    const int S = bot_slices(c01);
    for (int cs = threadIdx.x; cs < c01 * S; cs += blockDim.x) {
        const int sl = cs / c01, col = cs - sl * c01;
        const int cj = col / C.n[0], cix = col - cj * C.n[0];
        for (int ck = sl; ck < C.n[2]; ck += S) {
            const int lin = col + ck * c01;
            const int ci[3] = {cix, cj, ck};
            int fb[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) fb[a] = crs[a] ? 2 * ci[a] - (face[a] ? 1 : 0) : ci[a];
            // every window point lies in the fine grid after wrapping: load all 27
            T v[27];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 3; ++ii)
                        v[ii + 3 * jj + 9 * kk] = rf[wrap(fb[0] + ii, F.n[0]) + F.n[0] * wrap(fb[1] + jj, F.n[1]) +
                                                     f01 * wrap(fb[2] + kk, F.n[2])];
            T acc = (T)0;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 3; ++ii)
                        if (kk < fc[2] && jj < fc[1] && ii < fc[0])
                            acc = fmad(restrict_weight<T>(crs[0], face[0], ii) *
                                           restrict_weight<T>(crs[1], face[1], jj) *
                                           restrict_weight<T>(crs[2], face[2], kk),
                                       v[ii + 3 * jj + 9 * kk], acc);
            bc[lin] = pinned(comp, ci, R.bc) ? (T)0 : acc;
        }
    }
}

// x_f += P x_c over the fine level: the eight coarse values of each point are
// loaded at valid indices and the terms prolong_at would sum are added in its order
template <typename T>
__device__ __forceinline__ void bot_prolong(const RepDev &R, const LevDev &F, const LevDev &C, int comp,
                                            const T *xc, T *xf) {
    const int f01 = F.n[0] * F.n[1];
    const int c01 = C.n[0] * C.n[1];
    const int S = bot_slices(f01);
    for (int cs = threadIdx.x; cs < f01 * S; cs += blockDim.x) {
        const int sl = cs / f01, col = cs - sl * f01;
        const int fj = col / F.n[0], fix = col - fj * F.n[0];
        const ProlongAxis<T> px = prolong_axis<T>(fix, F.n[0], C.n[0], R.bc[0], comp == 0, comp);
        const ProlongAxis<T> py = prolong_axis<T>(fj, F.n[1], C.n[1], R.bc[1], comp == 1, comp);
        const int xi1 = px.cnt > 1 ? px.i1 : px.i0, yi1 = py.cnt > 1 ? py.i1 : py.i0;
        for (int fk = sl; fk < F.n[2]; fk += S) {
            const int fi[3] = {fix, fj, fk};
            const ProlongAxis<T> pz = prolong_axis<T>(fk, F.n[2], C.n[2], R.bc[2], comp == 2, comp);
            const int zi1 = pz.cnt > 1 ? pz.i1 : pz.i0;
            T v[8];
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii)
                        v[ii + 2 * jj + 4 * kk] = xc[(ii ? xi1 : px.i0) + C.n[0] * (jj ? yi1 : py.i0) +
                                                     c01 * (kk ? zi1 : pz.i0)];
            const int lin = col + fk * f01;
            const T old = xf[lin];
            T acc = (T)0;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                    for (int ii = 0; ii < 2; ++ii)
                        if (kk < pz.cnt && jj < py.cnt && ii < px.cnt)
                            acc = fmad((ii ? px.w1 : px.w0) * (jj ? py.w1 : py.w0) * (kk ? pz.w1 : pz.w0),
                                       v[ii + 2 * jj + 4 * kk], acc);
            if (!pinned(comp, fi, R.bc)) xf[lin] = old + acc;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(MGB_THREADS) void k_mg_bottom(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                           int c0, int nu, SweepW sw, const T *__restrict__ bpool,
                                                           T *xpool, T *tpool, unsigned res_t_mask,
                                                           const long long *coff, const T *__restrict__ Ainv,
                                                           const int *__restrict__ mask) {
    const BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev *lv = levs + be.rep * RB_MAXLEV;
    const int lb = R.lb, lc = R.nlev - 1;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sm = reinterpret_cast<T *>(smem_raw);
    auto xl = [&](int l) {
        long long o = 0;
        for (int k = lb; k < l; ++k) o += 2 * lv[k].N;
        return sm + o;
    };
    auto bl = [&](int l) { return xl(l) + lv[l].N; };
    T *t = xl(lc + 1);
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    {
        const T *src = bpool + lv[lb].off + comp * lv[lb].N;
        T *b = bl(lb);
        for (int i = threadIdx.x; i < (int)lv[lb].N; i += blockDim.x) b[i] = src[i];
    }
    __syncthreads();
    for (int l = lb; l < lc; ++l) {
        T *x = xl(l), *b = bl(l);
        for (int k = 1; k <= nu; ++k) {
            T *out = ((nu - k) % 2 == 0) ? x : t;
            T *in = (out == x) ? t : x;
            if (k == 1) bot_sweep<T, MG_FIRST>(R, lv[l], comp, s, (T)sw.w[k - 1], in, out, b);
            else bot_sweep<T, MG_SWEEP>(R, lv[l], comp, s, (T)sw.w[k - 1], in, out, b);
            __syncthreads();
        }
        bot_sweep<T, MG_RESID>(R, lv[l], comp, s, (T)0, x, t, b);
        __syncthreads();
        bot_restrict<T>(R, lv[l], lv[l + 1], comp, t, bl(l + 1));
        __syncthreads();
    }
    {
        const int m = (int)lv[lc].N;
        const T *A = Ainv + coff[be.rep * 4 + comp];
        const T *b = bl(lc);
        T *x = xl(lc);
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            T acc = (T)0;
            const T *row = A + (long long)i * m;
            for (int j = 0; j < m; ++j) acc = fmad(row[j], b[j], acc);
            x[i] = acc;
        }
        __syncthreads();
    }
    const T *res = xl(lc);
    for (int l = lc - 1; l >= lb; --l) {
        T *x = xl(l);
        const LevDev &F = lv[l], &C = lv[l + 1];
        bot_prolong<T>(R, F, C, comp, res, x);
        __syncthreads();
        T *in = x, *out = t;
        for (int k = 1; k <= nu; ++k) {
            bot_sweep<T, MG_SWEEP>(R, F, comp, s, (T)sw.w[k - 1], in, out, bl(l));
            __syncthreads();
            T *tmp = in; in = out; out = tmp;
        }
        res = in;
    }
    T *dst = (((res_t_mask >> lb) & 1u) ? tpool : xpool) + lv[lb].off + comp * lv[lb].N;
    for (int i = threadIdx.x; i < (int)lv[lb].N; i += blockDim.x) dst[i] = res[i];
}

template <typename T>
void launch_mg_bottom(Ctx &c, int c0, int nc, int nu, const SweepW &w, const T *b, T *x, T *t, unsigned res_t_mask) {
    if (c.n_tab_bot == 0) return;
    const size_t sh = sizeof(T) == 4 ? c.bot_lds32 : c.bot_lds64;
    hipLaunchKernelGGL(k_mg_bottom<T>, dim3(c.n_tab_bot, nc), dim3(MGB_THREADS), sh, c.stream, c.d_reps, c.d_levs,
                       c.d_tab_bot, c0, nu, w, b, x, t, res_t_mask, c.d_coarse_off, coarse_pool<T>(c), c.mask);
}
template void launch_mg_bottom<float>(Ctx &, int, int, int, const SweepW &, const float *, float *, float *, unsigned);
template void launch_mg_bottom<double>(Ctx &, int, int, int, const SweepW &, const double *, double *, double *,
                                       unsigned);

// ------------------------------------------------------------------ projection step
// d = D x* + r_pi ;  b_p (level 0) = -d  (so that -L phi = -d) ;  z_pi = -eta d.
// div sums the three axes in order with fused multiply-adds in both paths.
__device__ __forceinline__ void proj_div_out(double div, double rp, double f, double eta, float &bp, double &zp) {
    const double d = fmad(rp, f, div);
    bp = (float)(-d);
    zp = -eta * d;
}

// (r_pi is read as r * f, f = rs[rep * rstride], 1 without rs)
template <typename T, typename TZ>
__global__ void k_proj_div(const RepDev *reps, const LevDev *levs, const BlockEnt *tab, const T *__restrict__ xv,
                           const double *__restrict__ r, T *__restrict__ bp, TZ *__restrict__ z, const int *__restrict__ mask,
                           const double *__restrict__ rs, int rstride) {
    BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    const LevDev &Lv = levs[be.rep * RB_MAXLEV];
    const long long N = R.N;
    const double f = rs ? rs[(long long)be.rep * rstride] : 1.0;
    if constexpr (sizeof(T) == 4) {
        if (cells_row4(be, R, r) && cells_row4(be, R, z)) {
            const long long g0 = be.start + 4LL * threadIdx.x;
            if (g0 >= N) return;
            const int lin = (int)g0, n0 = R.n[0], n01 = R.n[0] * R.n[1];
            int idx[3];
            unlin(lin, R, idx);
            const float *u0 = (const float *)xv + Lv.off, *u1 = u0 + Lv.N, *u2 = u1 + Lv.N;
            // x: the four faces and the one after them
            const float4 a0 = ld_f4(u0 + lin);
            float after;
            if (idx[0] + 4 < n0) after = u0[lin + 4];
            else after = (R.bc[0] == RBFIB_PERIODIC) ? u0[lin + 4 - n0] : 0.f;
            // y and z: this row and the next (wrapped, or zero beyond a wall)
            const float4 a1 = ld_f4(u1 + lin), a2 = ld_f4(u2 + lin);
            float4 h1 = make_float4(0.f, 0.f, 0.f, 0.f), h2 = h1;
            if (idx[1] + 1 < R.n[1]) h1 = ld_f4(u1 + lin + n0);
            else if (R.bc[1] == RBFIB_PERIODIC) h1 = ld_f4(u1 + lin - (R.n[1] - 1) * n0);
            if (idx[2] + 1 < R.n[2]) h2 = ld_f4(u2 + lin + n01);
            else if (R.bc[2] == RBFIB_PERIODIC) h2 = ld_f4(u2 + lin - (R.n[2] - 1) * n01);
            const double *rp = r + R.off + 3 * N + lin;
            const double2 r01 = ld_d2(rp), r23 = ld_d2(rp + 2);
            const float x0[5] = {a0.x, a0.y, a0.z, a0.w, after};
            const float ys[4] = {a1.x, a1.y, a1.z, a1.w}, yh[4] = {h1.x, h1.y, h1.z, h1.w};
            const float zs[4] = {a2.x, a2.y, a2.z, a2.w}, zh[4] = {h2.x, h2.y, h2.z, h2.w};
            const double rr[4] = {r01.x, r01.y, r23.x, r23.y};
            const bool piny = R.bc[1] != RBFIB_PERIODIC && idx[1] == 0, pinz = R.bc[2] != RBFIB_PERIODIC && idx[2] == 0;
            float bo[4];
            double zo[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool pinx = R.bc[0] != RBFIB_PERIODIC && idx[0] + q == 0;
                double div = 0.0;
                div = fmad((double)x0[q + 1] - (pinx ? 0.0 : (double)x0[q]), R.inv_h, div);
                div = fmad((double)yh[q] - (piny ? 0.0 : (double)ys[q]), R.inv_h, div);
                div = fmad((double)zh[q] - (pinz ? 0.0 : (double)zs[q]), R.inv_h, div);
                proj_div_out(div, rr[q], f, R.eta, bo[q], zo[q]);
            }
            *reinterpret_cast<float4 *>((float *)bp + Lv.off + 3 * Lv.N + lin) = make_float4(bo[0], bo[1], bo[2], bo[3]);
            st_four(z + R.off + 3 * N + lin, zo);
            return;
        }
    }
    for (int t_ = 0; t_ < be.npt; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    if (lin >= N) continue;
    int idx[3];
    unlin(lin, R, idx);
    double div = 0.0;
    long long stride = 1;
    for (int c = 0; c < 3; ++c) {
        const T *u = xv + Lv.off + c * Lv.N;
        double lo = pinned(c, idx, R.bc) ? 0.0 : (double)u[lin];
        double hi;
        if (idx[c] + 1 < R.n[c]) hi = (double)u[lin + stride];
        else hi = (R.bc[c] == RBFIB_PERIODIC) ? (double)u[lin - (long long)(R.n[c] - 1) * stride] : 0.0;
        div = fmad(hi - lo, R.inv_h, div);
        stride *= R.n[c];
    }
    const double d = fmad(r[R.off + 3 * N + lin], f, div);
    bp[Lv.off + 3 * Lv.N + lin] = (T)(-d);
    z[R.off + 3 * N + lin] = (TZ)(-R.eta * d);
    }
}

template <typename T, typename TZ>
void launch_proj_div(Ctx &c, const T *xv, const double *r, T *bp, TZ *z, const double *rs) {
    hipLaunchKernelGGL((k_proj_div<T, TZ>), dim3(c.n_tab_cells), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_levs,
                       c.d_tab_cells, xv, r, bp, z, c.mask, rs, c.m + 1);
}

// z_v = x* - G phi  (phi in the pressure slot of the level-0 pool).
template <typename T, typename TZ>
__global__ void k_proj_correct(const RepDev *reps, const LevDev *levs, const BlockEnt *tab, const T *__restrict__ xv,
                               const T *__restrict__ phi, TZ *__restrict__ z, const int *__restrict__ mask) {
    BlockEnt be = tab[xcd_block(blockIdx.x, gridDim.x)];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    const LevDev &Lv = levs[be.rep * RB_MAXLEV];
    const long long N = R.N;
    if constexpr (sizeof(T) == 4) {
        if (cells_row4(be, R, z)) {
            const long long g0 = be.start + 4LL * threadIdx.x;
            if (g0 >= N) return;
            const int lin = (int)g0, n0 = R.n[0], n01 = R.n[0] * R.n[1];
            int idx[3];
            unlin(lin, R, idx);
            const float *ph = (const float *)phi + Lv.off + 3 * Lv.N;
            const float4 p4 = ld_f4(ph + lin);
            const float before = ph[lin + (idx[0] > 0 ? -1 : n0 - 1)];
            const float4 py = ld_f4(ph + lin + (idx[1] > 0 ? -n0 : (R.n[1] - 1) * n0));
            const float4 pz = ld_f4(ph + lin + (idx[2] > 0 ? -n01 : (R.n[2] - 1) * n01));
            const float pc[4] = {p4.x, p4.y, p4.z, p4.w};
            const float pmx[4] = {before, p4.x, p4.y, p4.z};
            const float pmy[4] = {py.x, py.y, py.z, py.w}, pmz[4] = {pz.x, pz.y, pz.z, pz.w};
            const bool piny = R.bc[1] != RBFIB_PERIODIC && idx[1] == 0, pinz = R.bc[2] != RBFIB_PERIODIC && idx[2] == 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 x4 = ld_f4((const float *)xv + Lv.off + c * Lv.N + lin);
                const float xs[4] = {x4.x, x4.y, x4.z, x4.w};
                double o[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool pin = c == 0 ? (R.bc[0] != RBFIB_PERIODIC && idx[0] + q == 0) : (c == 1 ? piny : pinz);
                    const float pm = c == 0 ? pmx[q] : (c == 1 ? pmy[q] : pmz[q]);
                    o[q] = pin ? 0.0 : fmad(-((double)pc[q] - (double)pm), R.inv_h, (double)xs[q]);
                }
                st_four(z + R.off + c * N + lin, o);
            }
            return;
        }
    }
    for (int t_ = 0; t_ < be.npt; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    if (lin >= N) continue;
    int idx[3];
    unlin(lin, R, idx);
    const T *ph = phi + Lv.off + 3 * Lv.N;
    double pc = (double)ph[lin];
    long long stride = 1;
    for (int c = 0; c < 3; ++c) {
        double out = 0.0;
        if (!pinned(c, idx, R.bc)) {
            double pm = (idx[c] > 0) ? (double)ph[lin - stride] : (double)ph[lin + (long long)(R.n[c] - 1) * stride];
            out = fmad(-(pc - pm), R.inv_h, (double)xv[Lv.off + c * Lv.N + lin]);
        }
        z[R.off + c * N + lin] = (TZ)out;
        stride *= R.n[c];
    }
    }
}

template <typename T, typename TZ>
void launch_proj_correct(Ctx &c, const T *xv, const T *phi, TZ *z) {
    hipLaunchKernelGGL((k_proj_correct<T, TZ>), dim3(c.n_tab_cells), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_levs,
                       c.d_tab_cells, xv, phi, z, c.mask);
}

// ------------------------------------------------------------------ fluctuating stress
// f_c(face) = scale * (DT W)_c = scale * [ (W_cc(cell f) - W_cc(cell f-1)) / h
//            + sum_{b != c} (w(n+1) W_cb(node n+1) - w(n) W_cb(node n)) / h ]
// where n is the cell index of the face along b and w = sqrt(2) on wall nodes.
__device__ __forceinline__ int fam_index(int c, int b) {
    if (c == b) return c;
    // order: xy, xz, yx, yz, zx, zy
    return 3 + 2 * c + ((b > c) ? b - 1 : b);
}

__device__ __forceinline__ double noise_W(uint64_t seed, uint64_t step, const RepDev &R, const long long *fam_off,
                                          int fam, int c, int b, int i, int j, int k) {
    int dims[3] = {R.n[0], R.n[1], R.n[2]};
    if (b != c && R.bc[b] != RBFIB_PERIODIC) dims[b] += 1;
    long long lin = (long long)i + (long long)dims[0] * ((long long)j + (long long)dims[1] * k);
    return philox_normal(seed, 1u, step, (uint64_t)(fam_off[fam] + lin));
}

__global__ void k_noise(const RepDev *reps, const BlockEnt *tab, double scale_base, uint64_t seed, uint64_t step,
                        double *__restrict__ f, int add) {
    BlockEnt be = tab[blockIdx.x];
    const RepDev &R = reps[be.rep];
    for (int t_ = 0; t_ < be.npt; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    long long N = R.N;
    if (lin >= N) continue;
    int idx[3];
    unlin(lin, R, idx);
    uint64_t rseed = seed + (uint64_t)be.rep;
    long long fam_off[10];
    fam_off[0] = 0;
    const int FC[9] = {0, 1, 2, 0, 0, 1, 1, 2, 2};
    const int FB[9] = {0, 1, 2, 1, 2, 0, 2, 0, 1};
    for (int q = 0; q < 9; ++q) {
        long long sz = 1;
        for (int a = 0; a < 3; ++a) sz *= (long long)R.n[a] + ((a == FB[q] && FB[q] != FC[q] && R.bc[a] != RBFIB_PERIODIC) ? 1 : 0);
        fam_off[q + 1] = fam_off[q] + sz;
    }
    double scale = scale_base * sqrt(R.eta / R.dV);
    const double SQ2 = 1.4142135623730951;
    for (int c = 0; c < 3; ++c) {
        double out = 0.0;
        if (!pinned(c, idx, R.bc)) {
            // family (c, c): cells idx and idx - e_c
            int im[3] = {idx[0], idx[1], idx[2]};
            im[c] -= 1;
            if (im[c] < 0) im[c] += R.n[c];   // only reachable on periodic axes
            double wp = noise_W(rseed, step, R, fam_off, fam_index(c, c), c, c, idx[0], idx[1], idx[2]);
            double wm = noise_W(rseed, step, R, fam_off, fam_index(c, c), c, c, im[0], im[1], im[2]);
            out += (wp - wm) * R.inv_h;
            for (int b = 0; b < 3; ++b) {
                if (b == c) continue;
                int fam = fam_index(c, b);
                int nb_ = idx[b];
                int np = nb_ + 1;
                double wlo = 1.0, whi = 1.0;
                int pi3[3] = {idx[0], idx[1], idx[2]};
                if (R.bc[b] != RBFIB_PERIODIC) {
                    // wall edges: sqrt(2) at a no-slip wall, 0 at a free-slip wall (no
                    // tangential stress), so that DT DT^T = -Lm with either ghost rule
                    const double ww = R.bc[b] == RBFIB_WALL ? SQ2 : 0.0;
                    if (nb_ == 0) wlo = ww;
                    if (np == R.n[b]) whi = ww;
                } else if (np == R.n[b]) np = 0;
                double Wlo = noise_W(rseed, step, R, fam_off, fam, c, b, pi3[0], pi3[1], pi3[2]);
                pi3[b] = np;
                double Whi = noise_W(rseed, step, R, fam_off, fam, c, b, pi3[0], pi3[1], pi3[2]);
                out += (whi * Whi - wlo * Wlo) * R.inv_h;
            }
            out *= scale;
        }
        double *dst = f + R.off + c * N + lin;
        if (add) *dst += out; else *dst = out;
    }
    if (!add) f[R.off + 3 * N + lin] = 0.0;
    }
}

void launch_noise(Ctx &c, double kT, double dt, uint64_t seed, uint64_t step, double *f, bool add) {
    double scale_base = sqrt(2.0 * kT / dt);
    hipLaunchKernelGGL(k_noise, dim3(c.n_tab_cells), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_cells, scale_base,
                       seed, step, f, add ? 1 : 0);
}

// Sliding walls: f_c += 2 eta U_w / h^2 on tangential faces adjacent to the wall.
__global__ void k_wall_rhs(const RepDev *reps, const BlockEnt *tab, double *__restrict__ f) {
    BlockEnt be = tab[blockIdx.x];
    const RepDev &R = reps[be.rep];
    if (!R.movwall) return;
    for (int t_ = 0; t_ < be.npt; ++t_) {
    long long lin = be.start + threadIdx.x + (long long)t_ * RB_BLOCK;
    long long N = R.N;
    if (lin >= N) continue;
    int idx[3];
    unlin(lin, R, idx);
    for (int c = 0; c < 3; ++c) {
        if (pinned(c, idx, R.bc)) continue;
        double add = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (a == c || R.bc[a] != RBFIB_WALL) continue;
            if (idx[a] == 0) add += 2.0 * R.eta * R.wv[a][0][c] * R.inv_h * R.inv_h;
            if (idx[a] == R.n[a] - 1) add += 2.0 * R.eta * R.wv[a][1][c] * R.inv_h * R.inv_h;
        }
        f[R.off + c * N + lin] += add;
    }
    }
}

void launch_wall_rhs(Ctx &c, double *f) {
    hipLaunchKernelGGL(k_wall_rhs, dim3(c.n_tab_cells), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_cells, f);
}

// explicit instantiations
template void launch_to_level0<float>(Ctx &, const double *, float *, int, int, const double *);
template void launch_to_level0<double>(Ctx &, const double *, double *, int, int, const double *);
template void launch_smooth<float>(Ctx &, int, int, int, const float *, float *, const float *, bool, double);
template void launch_smooth<double>(Ctx &, int, int, int, const double *, double *, const double *, bool, double);
template bool launch_smooth_first2<float>(Ctx &, int, int, int, float *, const float *, double, double);
template bool launch_smooth_first2<double>(Ctx &, int, int, int, double *, const double *, double, double);
template void launch_restrict<float>(Ctx &, int, int, int, const float *, const float *, float *, float *);
template void launch_restrict<double>(Ctx &, int, int, int, const double *, const double *, double *, double *);
template void launch_prolong<float>(Ctx &, int, int, int, const float *, float *);
template void launch_prolong<double>(Ctx &, int, int, int, const double *, double *);
template void launch_coarse<float>(Ctx &, int, int, int, const float *, float *);
template void launch_coarse<double>(Ctx &, int, int, int, const double *, double *);
template void launch_proj_div<float, double>(Ctx &, const float *, const double *, float *, double *, const double *);
template void launch_proj_div<float, float>(Ctx &, const float *, const double *, float *, float *, const double *);
template void launch_proj_div<double, double>(Ctx &, const double *, const double *, double *, double *,
                                              const double *);
template void launch_proj_correct<float, double>(Ctx &, const float *, const float *, double *);
template void launch_proj_correct<float, float>(Ctx &, const float *, const float *, float *);
template void launch_proj_correct<double, double>(Ctx &, const double *, const double *, double *);

}  // namespace rb

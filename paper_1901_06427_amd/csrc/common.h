// Internal declarations of the RB-FIB HIP library (gfx950).
//
// Layout of a packed state vector per replica r (offsets in RepDev):
//   off + 0*N .. : u_x  (N = nx*ny*nz slots, x fastest; slot i_x = 0 is the wall
//                        face when x is a wall axis and always holds 0)
//   off + 1*N .. : u_y,  off + 2*N : u_z,  off + 3*N : pi (cell centred)
//   off + 4*N .. : lambda [nm, 3],  then U [nb, 6]
// Multigrid level arrays hold the same four fields (u_x, u_y, u_z, pi) per level
// in FP32 or FP64, component c at  level_off + c * N_level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
#include <string>

#include "../../include/rbfib.h"

#define RB_MAXLEV 12
#define RB_TILE 4
#define RB_BLOCK 256
#define RB_CHUNK 1024          // default Krylov elements per block (RB_BLOCK * 4); the launch-geometry
                               // table chooses 512, 1024 or 2048 per workload class
// Fused multigrid kernels: a workgroup owns MGF_OX x MGF_OY x MGF_ZC fine points
// of one component (all even, so that coarse cells never straddle two blocks).
#define MGF_OX 32
#define MGF_OY 8
#define MGF_ZC 16
// A level runs fused only with at least this many workgroups (each marches
// through its z planes, so it needs several resident workgroups per CU).
#define MGF_MIN_BLOCKS 1024
// z-marching fluid apply: x-y tile edge (workgroup RB_AZT^2 threads)
#define RB_AZT 16
#define RB_NTIMING 7           // timing classes: apply, smoother sweep, fused down, fused up (level 0),
                               // Krylov dots, Krylov update, spreading of the apply
// LDS-resident bottom of the V-cycle: workgroup size and the largest LDS budget
// per workgroup an option may ask for
#define MGB_THREADS 512
#define MGB_LDS (64 * 1024)
// most damped-Jacobi sweeps per level and direction
#define RB_MAXSWEEP 16
// largest s-step Arnoldi block, and the packed upper triangle of its Gram matrix
#define RB_MAXS 4
#define RB_MAXG (RB_MAXS * (RB_MAXS + 1) / 2)

namespace rb {

// ---------------------------------------------------------------- descriptors
struct RepDev {
    int n[3];
    int bc[3];
    double h, inv_h, eta, dV;
    long long off;      // state offset of u_x
    long long N;        // cells
    long long len;      // state length 4N + 3nm + 6nb
    int nb, nm, b0, m0; // bodies/markers and their global first index
    int tdim[3];        // tile grid dims
    int tile0;          // first global tile index
    int nlev;
    int lb;             // first multigrid level run by the LDS bottom kernel (nlev - 1: coarsest only)
    int movwall;
    double wv[3][2][3];
    double inv_n0, inv_n01;   // 1/nx and 1/(nx*ny) for exact index splitting
};

// Descriptor of one replica with grid g and nb bodies of nm markers, its state at
// offset off, its first body, marker and tile b0, m0, tile0 (multigrid fields unset).
inline void rep_from_grid(RepDev &R, const rbfib_grid &g, int nb, int nm, long long off, int b0, int m0, int tile0) {
    R = RepDev();
    for (int a = 0; a < 3; ++a) { R.n[a] = g.n[a]; R.bc[a] = g.bc[a]; R.tdim[a] = (g.n[a] + RB_TILE - 1) / RB_TILE; }
    R.h = g.h; R.inv_h = 1.0 / g.h; R.eta = g.eta; R.dV = g.h * g.h * g.h;
    R.N = (long long)g.n[0] * g.n[1] * g.n[2];
    R.inv_n0 = 1.0 / g.n[0];
    R.inv_n01 = 1.0 / ((double)g.n[0] * g.n[1]);
    R.nb = nb; R.nm = nm; R.b0 = b0; R.m0 = m0;
    R.off = off;
    R.len = 4 * R.N + 3LL * nm + 6LL * nb;
    R.tile0 = tile0;
    R.movwall = 0;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 3; ++k) {
                const double v = (g.bc[a] == RBFIB_WALL && k != a) ? g.wall_vel[a][s][k] : 0.0;
                R.wv[a][s][k] = v;
                if (v != 0.0) R.movwall = 1;
            }
}

struct LevDev {
    int n[3];
    double inv_h2[3];   // 1/h_a^2 per axis at this level
    long long off;      // offset of this level's four fields in the level pool
    long long N;
    double inv_n0, inv_n01;
};

// (i, j, k) of a linear x-fastest index, without integer division: the quotient
// (lin + 1/2) / n is at least 1/(2n) away from an integer, so rounding the FP64
// product down is exact for every lin < 2^31.
__device__ __forceinline__ void split_index(long long lin, int n0, int n01, double inv_n0, double inv_n01, int idx[3]) {
    int l = (int)lin;
    int k = (int)(((double)l + 0.5) * inv_n01);
    int rem = l - k * n01;
    int j = (int)(((double)rem + 0.5) * inv_n0);
    idx[0] = rem - j * n0;
    idx[1] = j;
    idx[2] = k;
}

// ---------------------------------------------------------------- XCD-aware block order
// Workgroups are dispatched to the eight XCDs (each with its own L2) round-robin by
// blockIdx.x.  Stencil kernels read the neighbouring rows and planes of their
// chunk, so each XCD is given one contiguous range of table entries: table entry
// of workgroup b = (b mod 8) * (n / 8) + min(b mod 8, n mod 8) + b / 8, a
// permutation of [0, n).
#define RB_NXCD 8
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int x = b % RB_NXCD, i = b / RB_NXCD, per = n / RB_NXCD, rem = n % RB_NXCD;
    return x * per + min(x, rem) + i;
}

// ---------------------------------------------------------------- smoother arithmetic
// Every multigrid kernel evaluates the Laplacian, the Jacobi update, the residual
// and the transfer sums through these helpers, with explicit fused multiply-adds,
// so that the separate and the fused kernels round identically whatever the
// compiler's contraction choices.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc + (up - 2 self + um) ih2: one axis of the 7-point Laplacian
template <typename T>
__device__ __forceinline__ T lap_acc(T up, T self, T um, T ih2, T acc) {
    return fmad(fmad((T)-2, self, up) + um, ih2, acc);
}
// damped-Jacobi weight omega / (s diag)
template <typename T>
__device__ __forceinline__ T jacobi_w(T omega, T s, T dg) { return omega / (s * dg); }
// residual b - s lap
template <typename T>
__device__ __forceinline__ T mg_residual(T b, T s, T lap) { return fmad(-s, lap, b); }
// x + w (b - s lap)
template <typename T>
__device__ __forceinline__ T jacobi_step(T x, T b, T s, T lap, T w) { return fmad(mg_residual(b, s, lap), w, x); }
// ghost beyond a wall of a cell-centred quantity: even (pressure; tangential
// velocity at a free-slip wall) or odd (tangential velocity at a no-slip wall)
__device__ __forceinline__ bool even_ghost(int comp, int bc) { return comp == 3 || bc == RBFIB_SLIP; }

// diagonal term of axis a: -2, plus one ghost weight per wall the point touches
// (odd ghost: -1, even ghost: +1; face-normal axes have none)
template <typename T>
__device__ __forceinline__ T diag_axis(int comp, int a, int g, int n, int bc) {
    T da = (T)-2;
    if (bc != RBFIB_PERIODIC && a != comp) {
        const T gg = even_ghost(comp, bc) ? (T)1 : (T)-1;
        if (g == 0) da += gg;
        if (g == n - 1) da += gg;
    }
    return da;
}

// neighbour rules along one axis: 0 neighbour value, 1 zero (wall face),
// 2 even ghost (+self), 3 odd ghost (-self)
__device__ __forceinline__ int nbr_kind(int g, int d, int n, int bc, int a, int comp) {
    if (bc == RBFIB_PERIODIC) return 0;
    const int q = g + d;
    if (a == comp) return (q <= 0 || q >= n) ? 1 : 0;
    if (q < 0 || q >= n) return even_ghost(comp, bc) ? 2 : 3;
    return 0;
}

template <typename T>
__device__ __forceinline__ T pick(int kind, T nb, T self) {
    return kind == 0 ? nb : (kind == 1 ? (T)0 : (kind == 2 ? self : -self));
}

// ---------------------------------------------------------------- grid transfers
// Written with per-axis scalars (no dynamically indexed private arrays).
// Restriction weight of the o-th fine point along an axis.
template <typename T>
__device__ __forceinline__ T restrict_weight(bool coarsened, bool face, int o) {
    if (!coarsened) return (T)1;
    if (!face) return (T)0.5;
    return (o == 1) ? (T)0.5 : (T)0.25;
}

// Coarse points feeding one fine point along an axis: up to two (index, weight) pairs.
template <typename T>
struct ProlongAxis {
    int i0, i1, cnt;
    T w0, w1;
};

template <typename T>
__device__ __forceinline__ ProlongAxis<T> prolong_axis(int f, int nf, int nc, int bc, bool face, int comp) {
    ProlongAxis<T> p;
    if (nf == nc) { p.cnt = 1; p.i0 = p.i1 = f; p.w0 = (T)1; p.w1 = (T)0; return p; }
    const int I = f >> 1;
    if (face) {
        p.i0 = I; p.i1 = I;
        if ((f & 1) == 0) { p.cnt = 1; p.w0 = (T)1; p.w1 = (T)0; }
        else {
            p.cnt = 2; p.w0 = (T)0.5;
            int J = I + 1;
            T wj = (T)0.5;
            if (J >= nc) {
                if (bc == RBFIB_PERIODIC) J -= nc;
                else { J = I; wj = (T)0; }
            }
            p.i1 = J; p.w1 = wj;
        }
        if (bc != RBFIB_PERIODIC) {      // coarse face 0 on a wall axis is the wall
            if (p.i0 == 0) p.w0 = (T)0;
            if (p.cnt == 2 && p.i1 == 0) p.w1 = (T)0;
        }
    } else {
        p.cnt = 2; p.i0 = I; p.w0 = (T)0.75;
        int J = (f & 1) ? I + 1 : I - 1;
        T g = (T)0.25;
        if (J < 0 || J >= nc) {
            if (bc == RBFIB_PERIODIC) J = (J < 0) ? J + nc : J - nc;
            else { J = I; g = even_ghost(comp, bc) ? (T)0.25 : (T)-0.25; }
        }
        p.i1 = J; p.w1 = g;
    }
    return p;
}

// (P x_c) at fine point fi: face-normal axis linear (even faces copy, odd faces
// average), cell-centred axes (3/4, 1/4) with odd ghosts for velocity at walls and
// even ghosts for pressure.
template <typename T>
__device__ __forceinline__ T prolong_at(const RepDev &R, const LevDev &F, const LevDev &C, int comp, const int fi[3],
                                        const T *xc) {
    const ProlongAxis<T> px = prolong_axis<T>(fi[0], F.n[0], C.n[0], R.bc[0], comp == 0, comp);
    const ProlongAxis<T> py = prolong_axis<T>(fi[1], F.n[1], C.n[1], R.bc[1], comp == 1, comp);
    const ProlongAxis<T> pz = prolong_axis<T>(fi[2], F.n[2], C.n[2], R.bc[2], comp == 2, comp);
    T acc = (T)0;
    const long long c01 = (long long)C.n[0] * C.n[1];
    // fixed trip counts with predicates: all loads of the point issue together
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii)
                if (kk < pz.cnt && jj < py.cnt && ii < px.cnt)
                    acc = fmad((ii ? px.w1 : px.w0) * (jj ? py.w1 : py.w0) * (kk ? pz.w1 : pz.w0),
                               xc[(ii ? px.i1 : px.i0) + (long long)C.n[0] * (jj ? py.i1 : py.i0) +
                                  c01 * (kk ? pz.i1 : pz.i0)],
                               acc);
    return acc;
}

struct SweepW {         // weight of each smoothing sweep of a V-cycle (sweep k in w[k - 1])
    double w[RB_MAXSWEEP];
};

struct BlockEnt {       // one block of work: replica and local start index
    int rep;
    int npt;            // points per thread (stride RB_BLOCK): grid points for the stencil
                        // kernels, vector elements (chunk / RB_BLOCK) for the Krylov kernels
    long long start;
};

// Launch geometry of one context, from the table the autotuner writes (read at
// creation; built-in defaults without one): Krylov elements per workgroup,
// workgroups of the spreading grid-stride loop, (tile, marker) pairs staged per LDS
// round of the spreading pass, and grid points per thread of the multigrid and
// cell kernels (0: four on batches of at least 2^22 cells, else one).
struct Tuning {
    int krylov_chunk = RB_CHUNK;
    int spread_grid = 65536;
    int spread_p = 32;
    int mg_npt = 0;
    int apply_kc = -1;      // planes per workgroup of the z-marching apply; 0: two-cell kernel; -1: rule
};

struct ShapeDev {       // per distinct body shape: body-block preconditioner data
    int nm;
    long long minv_off; // (3nm)^2 doubles, body frame
    long long mk_off;   // (3nm) x 6 doubles: Minv K_ref
    long long n_off;    // 6x6 doubles: (K^T Minv K)^-1
    long long rref_off; // body-frame offsets (3nm doubles)
};

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ double phi4(double r) {
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) * 0.125;
    return 0.0;
}

__device__ __forceinline__ double dphi4(double r) {
    double a = fabs(r);
    double s = r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0);
    if (a <= 1.0) return s * (-2.0 + (4.0 - 8.0 * a) / (2.0 * sqrt(1.0 + 4.0 * a - 4.0 * a * a))) * 0.125;
    if (a < 2.0) return s * (-2.0 - (12.0 - 8.0 * a) / (2.0 * sqrt(-7.0 + 12.0 * a - 4.0 * a * a))) * 0.125;
    return 0.0;
}

// Fold a raw support index p along an axis of N cells.  normal: the axis is the
// face-normal axis of the velocity component.  Returns false when the point is a
// wall face (contributes nothing).  sgn is the sign of the reflection: -1 for the
// normal component and for a tangential one at a no-slip wall, +1 for a tangential
// one at a free-slip wall; cross = 0 (none), 1 (lower wall), 2 (upper wall).
// Indices are clamped into [0, N) so that even an invalid marker never addresses
// memory out of bounds.
__device__ __forceinline__ bool fold_index(int p, int N, int bc, bool normal, int &idx, double &sgn, int &cross) {
    sgn = 1.0;
    cross = 0;
    if (bc == RBFIB_PERIODIC) {
        int q = p % N;
        idx = q < 0 ? q + N : q;
        return true;
    }
    bool ok = true;
    if (normal) {
        if (p == 0 || p == N) ok = false;
        if (p < 0) { idx = -p; sgn = -1.0; cross = 1; }
        else if (p > N) { idx = 2 * N - p; sgn = -1.0; cross = 2; }
        else idx = p;
    } else {
        const double rs = bc == RBFIB_SLIP ? 1.0 : -1.0;
        if (p < 0) { idx = -1 - p; sgn = rs; cross = 1; }
        else if (p >= N) { idx = 2 * N - 1 - p; sgn = rs; cross = 2; }
        else idx = p;
    }
    if (idx < 0) { idx = 0; ok = false; }
    if (idx > N - 1) { idx = N - 1; ok = false; }
    return ok;
}

__device__ __forceinline__ void quat_to_R(const double *th, double R[9]) {
    double w = th[0], x = th[1], y = th[2], z = th[3];
    double xx = x * x, yy = y * y, zz = z * z;
    double xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0 - 2.0 * (yy + zz); R[1] = 2.0 * (xy - wz);       R[2] = 2.0 * (xz + wy);
    R[3] = 2.0 * (xy + wz);       R[4] = 1.0 - 2.0 * (xx + zz); R[5] = 2.0 * (yz - wx);
    R[6] = 2.0 * (xz - wy);       R[7] = 2.0 * (yz + wx);       R[8] = 1.0 - 2.0 * (xx + yy);
}

// Rotate(theta, phi): left-multiply by the unit quaternion of the rotation vector phi.
__device__ __forceinline__ void quat_rotate(const double *th, const double *phi, double *out) {
    double ang = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
    if (!(ang > 0.0)) { for (int k = 0; k < 4; ++k) out[k] = th[k]; return; }
    double s = sin(0.5 * ang) / ang, c = cos(0.5 * ang);
    double aw = c, ax = s * phi[0], ay = s * phi[1], az = s * phi[2];
    double bw = th[0], bx = th[1], by = th[2], bz = th[3];
    double w = aw * bw - (ax * bx + ay * by + az * bz);
    double x = aw * bx + bw * ax + (ay * bz - az * by);
    double y = aw * by + bw * ay + (az * bx - ax * bz);
    double z = aw * bz + bw * az + (ax * by - ay * bx);
    double nrm = sqrt(w * w + x * x + y * y + z * z);
    out[0] = w / nrm; out[1] = x / nrm; out[2] = y / nrm; out[3] = z / nrm;
}

// ---------------------------------------------------------------- Philox4x32-10
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

// Standard normal number `index` of (seed, stream, step) by Box-Muller.
__device__ __forceinline__ double philox_normal(uint64_t seed, uint32_t stream, uint64_t step, uint64_t index) {
    uint64_t pair = index >> 1;
    uint32_t c[4] = {(uint32_t)pair, stream, (uint32_t)step, (uint32_t)(step >> 32)};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint64_t a = ((((uint64_t)c[1]) << 32) | c[0]) >> 12;
    uint64_t b = ((((uint64_t)c[3]) << 32) | c[2]) >> 12;
    double u1 = ((double)a + 0.5) * 0x1p-52;
    double u2 = ((double)b + 0.5) * 0x1p-52;
    double rho = sqrt(-2.0 * log(u1));
    double ang = (2.0 * 3.141592653589793) * u2;
    return (index & 1) ? rho * sin(ang) : rho * cos(ang);
}

// ------------------------------------------------------------------ kernel weights
// Kernel of width W (4: Peskin's 4-point function; 6: the 6-point function of
// Bao, Kaiser & Peskin that the paper's runs use).  For a scaled coordinate s the W
// support points are base .. base + W - 1, base = floor(s) - (W/2 - 1), with weights
// phi(s - p).
//
// 6-point function: with x = s - floor(s) in [0, 1), its six values a_q = phi(x + 2 - q)
// satisfy five linear conditions (even and odd sums 1/2, moments 1 and 3 zero, moment 2
// K = 59/60 - sqrt(29)/20) and a quadratic one (sum of squares); solved in closed form
// they are polynomials in x plus multiples of t = a_5, the root of
// 28 t^2 + B(x) t + Cq(x) = 0 that vanishes at x = 0, taken as -2 Cq / (B + sqrt(disc))
// (no cancellation), disc = B^2 - 112 Cq.
#define RB_SQRT29 5.385164807134504
__device__ __forceinline__ void phi6_values(double x, double a[6]) {
    const double x2 = x * x, x3 = x2 * x, x4 = x2 * x2, x6 = x3 * x3;
    const double B = -7.0 / 3.0 * x3 - 1.5 * x2 + (0.45 + 0.35 * RB_SQRT29) * x + 0.075 * RB_SQRT29 + 0.775;
    const double Cq = 5.0 / 72.0 * x6 + (1.0 / 32.0 - RB_SQRT29 / 48.0) * x4;
    const double disc = B * B - 112.0 * Cq;
    const double t = -2.0 * Cq / (B + sqrt(disc));
    const double c0 = -RB_SQRT29 / 160.0 + 29.0 / 480.0;
    a[0] = t - x3 / 12.0 + x2 / 8.0 + (RB_SQRT29 - 13.0) / 80.0 * x + c0;
    a[1] = -3.0 * t + x3 / 6.0 - (7.0 + RB_SQRT29) / 40.0 * x + 0.25;
    a[2] = 2.0 * t - 0.25 * x2 + RB_SQRT29 / 80.0 + 91.0 / 240.0;
    a[3] = 2.0 * t - x3 / 6.0 + (7.0 + RB_SQRT29) / 40.0 * x + 0.25;
    a[4] = -3.0 * t + x3 / 12.0 + x2 / 8.0 + (13.0 - RB_SQRT29) / 80.0 * x + c0;
    a[5] = t;
}

// d a_q / dx, with t' from the quadratic: (56 t + B) t' = -(B' t + Cq'), 56 t + B = sqrt(disc)
__device__ __forceinline__ void dphi6_values(double x, double da[6]) {
    const double x2 = x * x, x3 = x2 * x, x4 = x2 * x2, x5 = x4 * x, x6 = x3 * x3;
    const double B = -7.0 / 3.0 * x3 - 1.5 * x2 + (0.45 + 0.35 * RB_SQRT29) * x + 0.075 * RB_SQRT29 + 0.775;
    const double Cq = 5.0 / 72.0 * x6 + (1.0 / 32.0 - RB_SQRT29 / 48.0) * x4;
    const double sq = sqrt(B * B - 112.0 * Cq);
    const double t = -2.0 * Cq / (B + sq);
    const double dB = -7.0 * x2 - 3.0 * x + 0.45 + 0.35 * RB_SQRT29;
    const double dCq = 5.0 / 12.0 * x5 + (1.0 / 8.0 - RB_SQRT29 / 12.0) * x3;
    const double dt = -(dB * t + dCq) / sq;
    da[0] = dt - 0.25 * x2 + 0.25 * x + (RB_SQRT29 - 13.0) / 80.0;
    da[1] = -3.0 * dt + 0.5 * x2 - (7.0 + RB_SQRT29) / 40.0;
    da[2] = 2.0 * dt - 0.5 * x;
    da[3] = 2.0 * dt - 0.5 * x2 + (7.0 + RB_SQRT29) / 40.0;
    da[4] = -3.0 * dt + 0.25 * x2 + 0.25 * x + (13.0 - RB_SQRT29) / 80.0;
    da[5] = dt;
}

// support base and the W weights phi(s - p), p = base + q
template <int W>
__device__ __forceinline__ int kernel_weights(double s, double w[W]);
template <>
__device__ __forceinline__ int kernel_weights<4>(double s, double w[4]) {
    const int b = (int)floor(s) - 1;
    for (int q = 0; q < 4; ++q) w[q] = phi4(s - (double)(b + q));
    return b;
}
template <>
__device__ __forceinline__ int kernel_weights<6>(double s, double w[6]) {
    const double f = floor(s);
    phi6_values(s - f, w);
    return (int)f - 2;
}
// the same with the derivatives d phi(s - p) / ds
template <int W>
__device__ __forceinline__ int kernel_weights_d(double s, double w[W], double dw[W]);
template <>
__device__ __forceinline__ int kernel_weights_d<4>(double s, double w[4], double dw[4]) {
    const int b = (int)floor(s) - 1;
    for (int q = 0; q < 4; ++q) { w[q] = phi4(s - (double)(b + q)); dw[q] = dphi4(s - (double)(b + q)); }
    return b;
}
template <>
__device__ __forceinline__ int kernel_weights_d<6>(double s, double w[6], double dw[6]) {
    const double f = floor(s);
    phi6_values(s - f, w);
    dphi6_values(s - f, dw);
    return (int)f - 2;
}

// 1-D folded weights of one marker coordinate for component c along axis a:
// raw support base..base+W-1, folded index and signed weight (0 when dropped).
template <int W>
__device__ __forceinline__ void axis_weights(const RepDev &R, double ra, int c, int a, int idx[W], double w[W],
                                             int cross[W]) {
    const double s = ra * R.inv_h - (a == c ? 0.0 : 0.5);
    double ph[W];
    const int b = kernel_weights<W>(s, ph);
    for (int q = 0; q < W; ++q) {
        int p = b + q;
        double sg;
        bool ok = fold_index(p, R.n[a], R.bc[a], a == c, idx[q], sg, cross[q]);
        w[q] = ok ? sg * ph[q] : 0.0;
    }
}

// (J u)_c from the cached 1-D weights and folded indices of marker m (layout
// [marker][component][axis][W]).
template <int W, typename TU>
__device__ __forceinline__ double interp_cached(const RepDev &R, const double *wc, const int *ic, int m, int c,
                                               const TU *u) {
    const double *w = wc + (long long)(3 * m + c) * 3 * W;
    const int *ix = ic + (long long)(3 * m + c) * 3 * W;
    double acc = 0.0;
    for (int z = 0; z < W; ++z) {
        double wz = w[2 * W + z];
        if (wz == 0.0) continue;
        for (int y = 0; y < W; ++y) {
            double wzy = wz * w[W + y];
            if (wzy == 0.0) continue;
            long long row = (long long)R.n[0] * ((long long)ix[W + y] + (long long)R.n[1] * ix[2 * W + z]);
            for (int x = 0; x < W; ++x) acc += wzy * w[x] * (double)u[row + ix[x]];
        }
    }
    return acc;
}

// Gradient with respect to the marker position of (J u)_c: the derivative along
// axis a replaces phi_a by phi_a' / h; fold signs and indices are fixed within each
// smooth piece of the kernel.
template <int W>
__device__ __forceinline__ void interp_grad(const RepDev &R, const double *rm, int c, const double *u, double g[3]) {
    int idx[3][W], cr[3][W];
    double w[3][W], dw[3][W];
    for (int a = 0; a < 3; ++a) {
        double s = rm[a] * R.inv_h - (a == c ? 0.0 : 0.5);
        double ph[W], dph[W];
        const int b = kernel_weights_d<W>(s, ph, dph);
        for (int q = 0; q < W; ++q) {
            int p = b + q;
            double sg;
            bool ok = fold_index(p, R.n[a], R.bc[a], a == c, idx[a][q], sg, cr[a][q]);
            w[a][q] = ok ? sg * ph[q] : 0.0;
            dw[a][q] = ok ? sg * dph[q] * R.inv_h : 0.0;
        }
    }
    g[0] = g[1] = g[2] = 0.0;
    for (int z = 0; z < W; ++z)
        for (int y = 0; y < W; ++y) {
            long long row = (long long)R.n[0] * ((long long)idx[1][y] + (long long)R.n[1] * idx[2][z]);
            for (int x = 0; x < W; ++x) {
                double v = u[row + idx[0][x]];
                g[0] += dw[0][x] * w[1][y] * w[2][z] * v;
                g[1] += w[0][x] * dw[1][y] * w[2][z] * v;
                g[2] += w[0][x] * w[1][y] * dw[2][z] * v;
            }
        }
}

// ---------------------------------------------------------------- host context
struct MarkerSet {
    double *r = nullptr;      // [nm, 3]
    double *d = nullptr;      // [nm, 3] = R r_ref
    int *tile = nullptr;      // [nm] global tile
    int *perm = nullptr;      // [nm] global marker ids sorted by tile
    int *tile_count = nullptr, *tile_start = nullptr, *tile_fill = nullptr;
    int *active = nullptr;    // [ntiles] compacted tiles that have spreading pairs
    int *n_active = nullptr;  // device scalar
    // spreading pairs (target tile, marker), by tile then marker id; capacity pair_cap
    int *pair_count = nullptr, *pair_start = nullptr, *pair_fill = nullptr;   // [ntiles]
    int *pair_m = nullptr, *pair_tile = nullptr;                              // [pair_cap]
    long long pair_cap = 0;
    double *wc = nullptr;     // [nm][3 comp][3 axis][W] folded signed 1-D kernel weights
    int *ic = nullptr;        // [nm][3][3][W] folded grid indices of those weights
};

struct Timing {
    bool on = false;
    std::vector<hipEvent_t> ev[RB_NTIMING];
    std::vector<double> ev_bytes[RB_NTIMING];   // algorithmic bytes of each recorded launch
    size_t used[RB_NTIMING] = {};
    double bytes[RB_NTIMING] = {};
    long long launches[RB_NTIMING] = {};
    double total_ms[RB_NTIMING] = {};
};

struct Ctx {
    hipStream_t stream = nullptr;        // library-owned stream (default priority) all work runs on
    hipStream_t user_stream = nullptr;   // caller's stream, ordered against ours with events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<hipGraphExec_t> graphs[2];   // one captured FGMRES iteration per (fluid_only, j)
    double graph_tol = -1.0;                 // tolerance baked into the captured graphs
    double *theta_int = nullptr;             // [nb, 4] orientation copy read by the preconditioner
    const int *mask = nullptr;               // replica mask for grid/body kernels (null = all)
    rbfib_opts opts;
    int nrep = 0;
    int kw = 4;               // delta-kernel width (4 or 6), fixed at creation
    Tuning tune;              // launch geometry, fixed at creation
    std::vector<RepDev> reps;
    long long L = 0;          // state length
    int nb = 0, nm = 0;
    int ntiles = 0;
    int maxlev = 0;
    int max_body_nm = 1;                 // largest marker count of one body
    std::vector<double> h_body_len;      // L_p per body (host copy)

    // device descriptors
    RepDev *d_reps = nullptr;
    LevDev *d_levs = nullptr;            // [nrep * RB_MAXLEV]
    std::vector<LevDev> levs;
    int *d_marker_body = nullptr, *d_body_rep = nullptr, *d_body_off = nullptr;  // body_off: [nb+1] global marker offsets
    int *d_tile_rep = nullptr;
    double *d_rref = nullptr;            // [nm, 3]
    int *d_body_shape = nullptr;
    ShapeDev *d_shapes = nullptr;
    double *d_shape_data = nullptr;
    double *d_body_len = nullptr;        // L_p
    double d_dummy = 0.0;

    // block tables
    BlockEnt *d_tab_cells = nullptr; int n_tab_cells = 0;         // level 0, all replicas, per cell chunk
    BlockEnt *d_tab_cells2 = nullptr; int n_tab_cells2 = 0;       // two cells per thread (apply)
    BlockEnt *d_tab_az = nullptr; int n_tab_az = 0;               // z-marching apply tiles (0: unused)
    int apply_kc = 0;                                             // their planes (0: two-cell apply)
    BlockEnt *d_tab_vec = nullptr; int n_tab_vec = 0;             // state chunks
    std::vector<int> vec_first, vec_nblk;                         // per replica block range
    int *d_vec_first = nullptr, *d_vec_nblk = nullptr;
    BlockEnt *d_tab_lev[RB_MAXLEV] = {nullptr};  int n_tab_lev[RB_MAXLEV] = {0};   // replicas with level l, not coarsest
    BlockEnt *d_tab_crs[RB_MAXLEV] = {nullptr};  int n_tab_crs[RB_MAXLEV] = {0};   // replicas whose coarsest is l
    BlockEnt *d_tab_all[RB_MAXLEV] = {nullptr};  int n_tab_all[RB_MAXLEV] = {0};   // replicas having level l
    // fused level kernels (start = tile index of level l), replicas that have level l+1
    BlockEnt *d_tab_mg[RB_MAXLEV] = {nullptr};   int n_tab_mg[RB_MAXLEV] = {0};
    // LDS bottom kernel: one entry per replica, dynamic LDS bytes in each precision
    BlockEnt *d_tab_bot = nullptr; int n_tab_bot = 0;
    size_t bot_lds32 = 0, bot_lds64 = 0;
    double lev_cells[RB_MAXLEV] = {0};   // points of level l summed over the replicas that have level l+1
    double lev_cells_c[RB_MAXLEV] = {0}; // points of level l+1 over the same replicas
    double cells_all = 0;                // level-0 points over all replicas
    int mg_npt = 1;                      // points per thread of the multigrid block tables
    bool lev_row4[RB_MAXLEV] = {false};  // every replica smoothed at level l has rows a multiple of 4 long
    // coarse dense inverses
    long long *d_coarse_off = nullptr;   // [nrep * 4] offset into coarse pools (doubles)
    double *d_coarse64 = nullptr;
    float *d_coarse32 = nullptr;
    int max_coarse = 0;

    // multigrid pools (x, b, t) in the chosen precision
    long long lev_total = 0;
    void *mg_x = nullptr, *mg_b = nullptr, *mg_t = nullptr;
    bool mg_fp32 = false;

    // marker sets: 0 = Q^n, 1 = Q+, 2 = Q-, 3 = new configuration
    MarkerSet ms[4];
    int *d_scan = nullptr;      // block sums of the tile scans
    int *d_flags = nullptr;     // [nrep]: bit 0 marker outside the domain, bit 1 bodies too close
    int *h_flags = nullptr;     // pinned host copy

    // Krylov
    int m = 0;
    double *V = nullptr, *Z = nullptr, *W = nullptr;
    float *Zf = nullptr;        // the preconditioned vectors in FP32 when the multigrid is FP32 (Z unused)
    double *xsol = nullptr, *rhs = nullptr;
    double *partial = nullptr;  // [n_tab_vec * (m+1)]
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *gv = nullptr, *beta0 = nullptr, *hcol = nullptr, *yv = nullptr;
    double *inv_nu = nullptr;   // [nrep][m+1]: basis vector i is stored as u_i, with v_i = inv_nu[i] u_i
    double *hblk = nullptr;     // [RB_MAXS][nrep][m+1]: projections of an s-step block's new vectors
    double *gram = nullptr;     // [nrep][RB_MAXG]: upper triangle of their Gram matrix
    double *tco = nullptr;      // [nrep][RB_MAXS][RB_MAXS]: combine coefficients R_lk / R_ll
    int *active = nullptr, *cyc_active = nullptr, *jf = nullptr, *status = nullptr, *iters = nullptr;
    int *h_count = nullptr;     // pinned
    double *d_resid = nullptr;  // [nrep]
    int *d_count = nullptr;
    long long *d_active_len = nullptr;   // timing runs: state length of the active replicas

    // SEM scratch
    double *q_buf[3] = {nullptr, nullptr, nullptr};      // q+, q-, q_new  [nb, 3]
    double *th_buf[3] = {nullptr, nullptr, nullptr};     // [nb, 4]
    double *Wf = nullptr, *Wt = nullptr, *WFT = nullptr, *Fp = nullptr, *slip_acc = nullptr, *UR = nullptr;
    // second-order SEM variants, kept between their predictor and corrector calls:
    // Q^n, the predictor Q*, and [U^n | U_det^n | U_det*] per body (6 each)
    double *trap_q0 = nullptr, *trap_th0 = nullptr, *trap_q = nullptr, *trap_th = nullptr, *trap_U = nullptr;
    bool trap_ready = false;
    double trap_dt = 0.0, trap_alpha = 1.0;
    std::vector<int> trap_status;
    double *jbc = nullptr;      // [nm, 3] scratch for the sliding-wall interpolation term
    double *xR = nullptr, *xS = nullptr;

    Timing timing;
};

// ---------------------------------------------------------------- launchers
// grid / multigrid (grid.hip)
template <typename TX> void launch_apply_fluid(Ctx &c, const TX *x, double *y);
template <typename T> void launch_to_level0(Ctx &c, const double *src, T *b, int c0, int nc, const double *rs = nullptr);
template <typename T> void launch_smooth(Ctx &c, int lev, int c0, int nc, const T *xin, T *xout, const T *b, bool first,
                                          double omega);
template <typename T> bool launch_smooth_first2(Ctx &c, int lev, int c0, int nc, T *xout, const T *b, double omega1,
                                                 double omega2);
template <typename T> void launch_restrict(Ctx &c, int lev, int c0, int nc, const T *x, const T *b, T *bc, T *r);
template <typename T> void launch_mg_bottom(Ctx &c, int c0, int nc, int nu, const SweepW &w, const T *b, T *x, T *t,
                                           unsigned res_t_mask);
template <typename T> void launch_prolong(Ctx &c, int lev, int c0, int nc, const T *xc, T *xf);
template <typename T> void launch_coarse(Ctx &c, int lev, int c0, int nc, const T *b, T *x);
// fused level kernels (mgfused.hip)
template <typename T> void launch_mg_down(Ctx &c, int lev, int c0, int nc, const T *b, T *x, double omega1, double omega2);
template <typename T> void launch_mg_up(Ctx &c, int lev, int c0, int nc, const T *b, const T *xin, const T *xc, T *xout,
                                       double omega1, double omega2);
template <typename T, typename TZ> void launch_proj_div(Ctx &c, const T *xv, const double *r, T *bp, TZ *z,
                                                       const double *rs = nullptr);
template <typename T, typename TZ> void launch_proj_correct(Ctx &c, const T *xv, const T *phi, TZ *z);
void launch_noise(Ctx &c, double kT, double dt, uint64_t seed, uint64_t step, double *f, bool add);
void launch_wall_rhs(Ctx &c, double *f);

// immersed boundary and bodies (ib.hip)
void launch_markers(Ctx &c, MarkerSet &ms, const double *q, const double *theta, bool counts_zeroed = false);
template <typename TL> void launch_spread(Ctx &c, MarkerSet &ms, const TL *lam, double *y, double alpha);
template <typename T, typename TL>
void launch_spread_level0(Ctx &c, MarkerSet &ms, const TL *lam, T *pool, double alpha);
template <typename TX> void launch_body_apply(Ctx &c, MarkerSet &ms, const double *q, const TX *x, double *y);
template <typename TZ>
void launch_body_precond(Ctx &c, MarkerSet &ms, const double *theta, const double *r, TZ *z,
                         const double *rs = nullptr);
void launch_interp(Ctx &c, MarkerSet &ms, const double *x, double *out, double alpha, bool accumulate);
void launch_interp_bc(Ctx &c, MarkerSet &ms, double *out, double alpha);
void launch_body_rfd(Ctx &c, double kT, double delta, uint64_t seed, uint64_t step, const double *q,
                     const double *theta);
void launch_rfd_terms(Ctx &c, double delta);
void launch_rfd_forces(Ctx &c, double delta, const double *FT);
void launch_set_rhs_U(Ctx &c, const double *Fp, double *b);
void launch_body_distance(Ctx &c, double dmin);
void launch_sem_rhs_lambda(Ctx &c, const double *slip, double *b);
void launch_update_positions(Ctx &c, const double *q, const double *theta, const double *U, double dt);
void launch_commit_positions(Ctx &c, double *q, double *theta);
void launch_body_grad(Ctx &c, const double *x, const double *xa, const double *theta, double *dFT, double *dq,
                      double *dphi, double *dtheta);
void launch_set_rhs_adjoint(Ctx &c, const double *Ubar, double *b);
void launch_copy_U(Ctx &c, const double *x, double *U, double scale);
void launch_rk2_update(Ctx &c, const double *q, const double *theta, const double *Uem, const double *Ud0,
                       const double *Ud1, double w, double dt, double *Uc);
void launch_body_forces(Ctx &c, const double *q, const double *theta, double phi0, double d, double b,
                        const double fconst[3], double *FT);
void launch_set_rhs(Ctx &c, const double *FT, const double *slip, double *b);

// Krylov (krylov.hip)
void launch_dots(Ctx &c, const double *V, int nvec, const double *w, double *out /*[nrep*(m+1)]*/, const int *mask,
                 const double *scale = nullptr);
void launch_axpy_multi(Ctx &c, const double *V, int nvec, const double *coef, double *w, double sign, const int *mask,
                       const double *scale = nullptr);
void launch_norm(Ctx &c, const double *w, double *out, const int *mask);
void launch_axpy_multi_norm(Ctx &c, const double *V, int nvec, const double *coef, double *w, double *nrm,
                            const int *mask, const double *scale = nullptr);
void launch_scale(Ctx &c, const double *w, const double *s, double *out, const int *mask, bool inverse);
void launch_axpby(Ctx &c, double a, const double *x, double b, const double *y, double *out, const int *mask);
void launch_copy(Ctx &c, const double *x, double *y, const int *mask);
void launch_zero(Ctx &c, double *y, const int *mask);
void launch_block_dots(Ctx &c, int S, const double *V, int nvec, const double *W, const int *mask,
                       const double *scale);
void launch_block_update(Ctx &c, int S, const double *V, int nvec, double *W, const int *mask, const double *scale);
void launch_givens_s(Ctx &c, int j, int S, double tol);
void launch_combine_s(Ctx &c, int S, double *W, const int *mask);
void launch_givens(Ctx &c, int j, double tol);
void launch_start_cycle(Ctx &c);
void launch_trisolve_update(Ctx &c);
template <typename TY> void launch_zero_bodies(Ctx &c, TY *y);   // zero the lambda and U slots

template <typename T> void zero_device(Ctx &c, T *p, long long n);

}  // namespace rb

#define HIP_OK(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) { rb_last_hip_error(e_, #expr, __FILE__, __LINE__); throw (int)RBFIB_EDEVICE; } } while (0)
void rb_last_hip_error(hipError_t e, const char *what, const char *file, int line);

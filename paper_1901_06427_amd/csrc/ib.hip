// Immersed-boundary and rigid-body kernels (paper Sec. III.B, III.C):
//   * marker geometry r_i = q_p + R(theta_p) r_i^ref and binning into 4^3-cell tiles;
//   * spreading S as a deterministic GATHER: per marker configuration, a list of
//     (tile, marker) pairs; per application one wavefront per tile projects its pairs'
//     cached kernel weights (4- or 6-point) onto the tile's 4-cell window per axis in
//     LDS and sums them in marker order, one lane per target cell -- no atomics;
//   * interpolation J fused with K U and K^T lambda, one workgroup per body;
//   * the per-body block of the preconditioner (dense body-frame blob mobility).
// Walls fold the kernel support by odd reflection so that J = dV S^* holds exactly.
#include "common.h"

namespace rb {

// ------------------------------------------------------------------ geometry
// The marker position is computed with contraction disabled and in a fixed
// operation order so that the integer cell/tile indices are reproducible.
__device__ void marker_pos(const double *q, const double *th, const double *rr, double d[3], double r[3]) {
#pragma clang fp contract(off)
    double w = th[0], x = th[1], y = th[2], z = th[3];
    double xx = x * x, yy = y * y, zz = z * z;
    double xy = x * y, xz = x * z, yz = y * z;
    double wx = w * x, wy = w * y, wz = w * z;
    double R0 = 1.0 - 2.0 * (yy + zz), R1 = 2.0 * (xy - wz), R2 = 2.0 * (xz + wy);
    double R3 = 2.0 * (xy + wz), R4 = 1.0 - 2.0 * (xx + zz), R5 = 2.0 * (yz - wx);
    double R6 = 2.0 * (xz - wy), R7 = 2.0 * (yz + wx), R8 = 1.0 - 2.0 * (xx + yy);
    double a = rr[0], b = rr[1], c = rr[2];
    double t0 = R0 * a, t1 = R1 * b, t2 = R2 * c;
    double t3 = R3 * a, t4 = R4 * b, t5 = R5 * c;
    double t6 = R6 * a, t7 = R7 * b, t8 = R8 * c;
    d[0] = (t0 + t1) + t2;
    d[1] = (t3 + t4) + t5;
    d[2] = (t6 + t7) + t8;
    r[0] = q[0] + d[0];
    r[1] = q[1] + d[1];
    r[2] = q[2] + d[2];
}

template <int W>
__global__ void k_markers(const RepDev *reps, const int *marker_body, const int *body_rep, const double *q,
                          const double *theta, const double *rref, int nm, double *r_out, double *d_out, int *tile,
                          int *tile_count, int *flags, double *wc, int *ic) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    int p = marker_body[m];
    const RepDev &R = reps[body_rep[p]];
    double d[3], r[3];
    marker_pos(q + 3 * p, theta + 4 * p, rref + 3 * m, d, r);
    // orientations must be unit quaternions to 1e-12 (bit 3 of the replica's flags)
    const double *th = theta + 4 * p;
    const double qn = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2] + th[3] * th[3]);
    if (!(fabs(qn - 1.0) <= 1e-12)) atomicOr(&flags[body_rep[p]], 8);
    int cell[3];
    bool outside = false;
    for (int a = 0; a < 3; ++a) {
        double s = r[a] * R.inv_h;
        if (!(s == s) || fabs(s) > 1e9) { outside = true; s = 0.0; }
        long long cc = (long long)floor(s);
        if (R.bc[a] == RBFIB_PERIODIC) {
            cc %= R.n[a];
            if (cc < 0) cc += R.n[a];
        } else {
            double L = (double)R.n[a] * R.h;
            if (!(r[a] > 0.0 && r[a] < L)) outside = true;
            if (cc < 0) cc = 0;
            if (cc > R.n[a] - 1) cc = R.n[a] - 1;
        }
        cell[a] = (int)cc;
    }
    int t = R.tile0 + (cell[0] >> 2) + R.tdim[0] * ((cell[1] >> 2) + R.tdim[1] * (cell[2] >> 2));
    for (int a = 0; a < 3; ++a) { r_out[3 * m + a] = r[a]; d_out[3 * m + a] = d[a]; }
    tile[m] = t;
    atomicAdd(&tile_count[t], 1);
    // 1-D folded kernel weights, reused by every spread and interpolation at this configuration
    for (int c = 0; c < 3; ++c)
        for (int a = 0; a < 3; ++a) {
            int idx[W], cr[W];
            double w[W];
            axis_weights<W>(R, r[a], c, a, idx, w, cr);
            long long o = ((long long)(3 * m + c) * 3 + a) * W;
            for (int k = 0; k < W; ++k) { wc[o + k] = w[k]; ic[o + k] = idx[k]; }
        }
    if (outside) atomicOr(&flags[body_rep[p]], 1);
}

// ------------------------------------------------------------------ scans over tiles
// Exclusive scan of n ints in three launches: sums of SCAN_B-entry blocks, one
// workgroup scanning the block sums, and each block's own scan plus its offset.
// pred = 1 scans (v > 0) instead of v and writes the indices with v > 0 to list
// (a stable compaction); otherwise out = the exclusive prefix and fill = 0.
#define SCAN_T 256
#define SCAN_B (4 * SCAN_T)

__device__ __forceinline__ int scan_val(const int *in, int i, int n, int pred) {
    if (i >= n) return 0;
    const int v = in[i];
    return pred ? (v > 0 ? 1 : 0) : v;
}

// exclusive scan of one value per thread across the workgroup (SCAN_T threads)
__device__ __forceinline__ int block_exscan(int v, int *sh, int &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_T; o <<= 1) {
        const int a = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[SCAN_T - 1];
    const int ex = sh[t] - v;
    __syncthreads();
    return ex;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_sums(const int *in, int n, int pred, int *bsum) {
    __shared__ int sh[SCAN_T];
    const int base = blockIdx.x * SCAN_B + 4 * threadIdx.x;
    int v = 0;
    for (int k = 0; k < 4; ++k) v += scan_val(in, base + k, n, pred);
    int total;
    block_exscan(v, sh, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the nb block sums in place; the grand total to *total
__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(int *bsum, int nb, int *total) {
    __shared__ int sh[SCAN_T];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += SCAN_T) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int tot;
        const int ex = block_exscan(v, sh, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_local(const int *in, int n, int pred, const int *boff, int *out,
                                                       int *fill, int *list) {
    __shared__ int sh[SCAN_T];
    const int base = blockIdx.x * SCAN_B + 4 * threadIdx.x;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) { v[k] = scan_val(in, base + k, n, pred); s += v[k]; }
    int total;
    int ex = boff[blockIdx.x] + block_exscan(s, sh, total);
    for (int k = 0; k < 4; ++k) {
        const int i = base + k;
        if (i < n) {
            if (pred) {
                if (v[k]) list[ex] = i;
            } else {
                out[i] = ex;
                if (fill) fill[i] = 0;
            }
        }
        ex += v[k];
    }
}

// start = exclusive scan of count, fill = 0
static void scan_tiles(Ctx &c, const int *count, int *start, int *fill) {
    const int nb = (c.ntiles + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_T), 0, c.stream, count, c.ntiles, 0, c.d_scan);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_T), 0, c.stream, c.d_scan, nb, (int *)nullptr);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_T), 0, c.stream, count, c.ntiles, 0, c.d_scan, start, fill,
                       (int *)nullptr);
}

// list = the tiles with count > 0 in order, *n_out = how many
static void compact_tiles(Ctx &c, const int *count, int *list, int *n_out) {
    const int nb = (c.ntiles + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_T), 0, c.stream, count, c.ntiles, 1, c.d_scan);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(SCAN_T), 0, c.stream, c.d_scan, nb, n_out);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(SCAN_T), 0, c.stream, count, c.ntiles, 1, c.d_scan,
                       (int *)nullptr, (int *)nullptr, list);
}

__global__ void k_tile_place(const int *tile, const int *start, int *fill, int *perm, int nm) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    int t = tile[m];
    int slot = start[t] + atomicAdd(&fill[t], 1);
    perm[slot] = m;
}

// insertion sort of each tile's entries by id: a stable (tile, id) order; entries at
// or beyond cap (never written) are left out
__global__ void k_tile_sort(const int *start, const int *count, int *perm, int ntiles, long long cap) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int b = start[t];
    int n = (int)min((long long)count[t], cap - b);
    for (int i = 1; i < n; ++i) {
        int v = perm[b + i];
        int j = i - 1;
        while (j >= 0 && perm[b + j] > v) { perm[b + j + 1] = perm[b + j]; --j; }
        perm[b + j + 1] = v;
    }
}

// ------------------------------------------------------------------ spreading pairs
// Spreading is built once per marker configuration as a list of (target tile,
// marker) pairs, sorted by tile and, within a tile, by marker id.  A marker pairs
// with every tile that holds, on each axis, a nonzero folded weight of one of its
// three staggered components.  The union of the three W-point supports along an
// axis covers at most W + 1 consecutive cells (wrapped on periodic axes, folded into
// the domain at walls), so it meets at most W/2 4-cell tiles, one more where a
// periodic axis ends in a partial tile.  The spreading kernel projects each pair's
// cached 1-D weights onto the tile's 4-cell window.
struct AxisTiles {
    int k = 0, t0 = 0, t1 = 0, t2 = 0, t3 = 0;   // scalars, not an array: no private memory
};

__device__ __forceinline__ void add_tile(AxisTiles &s, int t, bool &over) {
    if ((s.k > 0 && s.t0 == t) || (s.k > 1 && s.t1 == t) || (s.k > 2 && s.t2 == t) || (s.k > 3 && s.t3 == t)) return;
    if (s.k == 0) s.t0 = t;
    else if (s.k == 1) s.t1 = t;
    else if (s.k == 2) s.t2 = t;
    else if (s.k == 3) s.t3 = t;
    else { over = true; return; }
    ++s.k;
}

__device__ __forceinline__ int tile_at(const AxisTiles &s, int i) {
    return i == 0 ? s.t0 : (i == 1 ? s.t1 : (i == 2 ? s.t2 : s.t3));
}

template <int W>
__device__ __forceinline__ AxisTiles marker_axis_tiles(const double *wc, const int *ic, int m, int a, bool &over) {
    AxisTiles s;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const long long o = ((long long)(3 * m + c) * 3 + a) * W + q;
            if (wc[o] != 0.0) add_tile(s, ic[o] / RB_TILE, over);
        }
    return s;
}

// place = 0: count the pairs of each tile; place = 1: write them into the slots
// given by the exclusive scan of the counts (unordered within a tile).  A marker
// whose supports break the bound above (non-finite position) or a slot beyond the
// capacity flags its replica.
template <int W>
__global__ void k_pair_tiles(const RepDev *reps, const int *marker_body, const int *body_rep, const double *wc,
                             const int *ic, int nm, int place, int *pair_count, const int *pair_start, int *pair_fill,
                             int *pair_m, int *pair_tile, long long cap, int *flags) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm) return;
    const int rep = body_rep[marker_body[m]];
    const RepDev &R = reps[rep];
    bool over = false;
    const AxisTiles X = marker_axis_tiles<W>(wc, ic, m, 0, over);
    const AxisTiles Y = marker_axis_tiles<W>(wc, ic, m, 1, over);
    const AxisTiles Z = marker_axis_tiles<W>(wc, ic, m, 2, over);
    for (int z = 0; z < Z.k; ++z)
        for (int y = 0; y < Y.k; ++y)
            for (int x = 0; x < X.k; ++x) {
                const int t = R.tile0 + tile_at(X, x) + R.tdim[0] * (tile_at(Y, y) + R.tdim[1] * tile_at(Z, z));
                if (!place) {
                    atomicAdd(&pair_count[t], 1);
                } else {
                    const long long s = (long long)pair_start[t] + atomicAdd(&pair_fill[t], 1);
                    if (s < cap) { pair_m[s] = m; pair_tile[s] = t; }
                    else over = true;
                }
            }
    if (over) atomicOr(&flags[rep], 1);
}

template <int W>
static void markers_w(Ctx &c, MarkerSet &ms, const double *q, const double *theta, bool counts_zeroed) {
    if (!counts_zeroed) {
        HIP_OK(hipMemsetAsync(ms.tile_count, 0, sizeof(int) * c.ntiles, c.stream));
        HIP_OK(hipMemsetAsync(ms.pair_count, 0, sizeof(int) * c.ntiles, c.stream));
    }
    int nb = (c.nm + 255) / 256;
    if (c.nm > 0)
        hipLaunchKernelGGL(k_markers<W>, dim3(nb), dim3(256), 0, c.stream, c.d_reps, c.d_marker_body, c.d_body_rep, q,
                           theta, c.d_rref, c.nm, ms.r, ms.d, ms.tile, ms.tile_count, c.d_flags, ms.wc, ms.ic);
    scan_tiles(c, ms.tile_count, ms.tile_start, ms.tile_fill);
    if (c.nm > 0) {
        hipLaunchKernelGGL(k_tile_place, dim3(nb), dim3(256), 0, c.stream, ms.tile, ms.tile_start, ms.tile_fill,
                           ms.perm, c.nm);
        hipLaunchKernelGGL(k_tile_sort, dim3((c.ntiles + 255) / 256), dim3(256), 0, c.stream, ms.tile_start,
                           ms.tile_count, ms.perm, c.ntiles, (long long)c.nm);
        hipLaunchKernelGGL(k_pair_tiles<W>, dim3(nb), dim3(256), 0, c.stream, c.d_reps, c.d_marker_body, c.d_body_rep,
                           ms.wc, ms.ic, c.nm, 0, ms.pair_count, ms.pair_start, ms.pair_fill, ms.pair_m,
                           ms.pair_tile, ms.pair_cap, c.d_flags);
    }
    scan_tiles(c, ms.pair_count, ms.pair_start, ms.pair_fill);
    if (c.nm > 0) {
        hipLaunchKernelGGL(k_pair_tiles<W>, dim3(nb), dim3(256), 0, c.stream, c.d_reps, c.d_marker_body, c.d_body_rep,
                           ms.wc, ms.ic, c.nm, 1, ms.pair_count, ms.pair_start, ms.pair_fill, ms.pair_m,
                           ms.pair_tile, ms.pair_cap, c.d_flags);
        hipLaunchKernelGGL(k_tile_sort, dim3((c.ntiles + 255) / 256), dim3(256), 0, c.stream, ms.pair_start,
                           ms.pair_count, ms.pair_m, c.ntiles, ms.pair_cap);
    }
    compact_tiles(c, ms.pair_count, ms.active, ms.n_active);
}

// counts_zeroed: the caller has already cleared tile_count and pair_count (the
// allocation-free entry point does it in its set-up kernel instead of a memset).
void launch_markers(Ctx &c, MarkerSet &ms, const double *q, const double *theta, bool counts_zeroed) {
    if (c.kw == 6) markers_w<6>(c, ms, q, theta, counts_zeroed);
    else markers_w<4>(c, ms, q, theta, counts_zeroed);
}

// ------------------------------------------------------------------ spreading (gather)
// One wavefront per tile that has pairs, one lane per (x, y, z) cell of the tile.  The
// tile's pairs are taken SPREAD_P (16, 32 or 64) at a time: lane i loads the cached folded 1-D
// weights of pair i's marker (3 components x 3 axes x W points, with their folded
// indices) and its lambda, projects them onto the tile's 4-cell window on each axis
// (several support points can fold onto one cell next to a wall), folds lambda_c into
// the z factor, and leaves the 36 window weights in LDS; then every lane sums, for the
// three velocity components at once, the tensor-product weights of its cell over the
// staged pairs in marker order.  All loads of a round are independent, so a tile costs
// one round of latency per SPREAD_P pairs; the sum order is fixed (no atomics), so the
// result is deterministic.
// TO = double: y is a state vector (velocity of replica r at R.off + c N);
// with levs given: y is a multigrid pool, level 0 of each replica.
// the cached folded weights and indices of (marker m, component c, axis a)
template <int W>
__device__ __forceinline__ void load_axis(const double *__restrict__ wc, const int *__restrict__ ic, long long o,
                                          double w[W], int ix[W]);
template <>
__device__ __forceinline__ void load_axis<4>(const double *__restrict__ wc, const int *__restrict__ ic, long long o,
                                             double w[4], int ix[4]) {
    const double2 w01 = *reinterpret_cast<const double2 *>(wc + o);
    const double2 w23 = *reinterpret_cast<const double2 *>(wc + o + 2);
    const int4 i4 = *reinterpret_cast<const int4 *>(ic + o);
    w[0] = w01.x; w[1] = w01.y; w[2] = w23.x; w[3] = w23.y;
    ix[0] = i4.x; ix[1] = i4.y; ix[2] = i4.z; ix[3] = i4.w;
}
template <>
__device__ __forceinline__ void load_axis<6>(const double *__restrict__ wc, const int *__restrict__ ic, long long o,
                                             double w[6], int ix[6]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double2 wk = *reinterpret_cast<const double2 *>(wc + o + 2 * k);
        const int2 ik = *reinterpret_cast<const int2 *>(ic + o + 2 * k);
        w[2 * k] = wk.x; w[2 * k + 1] = wk.y;
        ix[2 * k] = ik.x; ix[2 * k + 1] = ik.y;
    }
}

template <typename TO, typename TL, int W, int SPREAD_P>
__global__ __launch_bounds__(64) void k_spread(const RepDev *reps, const int *tile_rep, const int *active,
                                               const int *n_active, const int *pair_start, const int *pair_count,
                                               long long cap, const int *__restrict__ pair_m,
                                               const double *__restrict__ wc, const int *__restrict__ ic,
                                               const TL *__restrict__ lam_state, TO *__restrict__ y,
                                               double alpha, const int *__restrict__ mask,
                                               const LevDev *__restrict__ levs) {
    __shared__ double sw[SPREAD_P * 36];
    const int lane = threadIdx.x;
    const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
    const int na = *n_active;
    // each XCD takes one contiguous range of the (spatially sorted) active tiles, so
    // the weights of a marker, which neighbouring tiles share, are fetched into one L2
    // (workgroup b runs on XCD b mod RB_NXCD); grids smaller than RB_NXCD stride plainly
    const int G = (int)gridDim.x;
    const bool split = G >= RB_NXCD;
    const int xcd = split ? (int)blockIdx.x % RB_NXCD : 0;
    const int lb = split ? (int)blockIdx.x / RB_NXCD : (int)blockIdx.x;
    const int nblk = split ? (G - xcd + RB_NXCD - 1) / RB_NXCD : G;
    const int t_beg = split ? (int)((long long)na * xcd / RB_NXCD) : 0;
    const int t_end = split ? (int)((long long)na * (xcd + 1) / RB_NXCD) : na;
    for (int it = t_beg + lb; it < t_end; it += nblk) {
        const int t = active[it];
        const int rep = tile_rep[t];
        if (mask && !mask[rep]) continue;
        const RepDev &R = reps[rep];
        const int lt = t - R.tile0;
        const int org[3] = {RB_TILE * (lt % R.tdim[0]), RB_TILE * ((lt / R.tdim[0]) % R.tdim[1]),
                            RB_TILE * (lt / (R.tdim[0] * R.tdim[1]))};
        const long long s0 = pair_start[t];
        const long long s1 = min(s0 + (long long)pair_count[t], cap);
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        for (long long base = s0; base < s1; base += SPREAD_P) {
            const int cnt = (int)min((long long)SPREAD_P, s1 - base);
            if (lane < cnt) {
                const int m = pair_m[base + lane];
                const TL *lam = lam_state + R.off + 4 * R.N + 3LL * (m - R.m0);
                double *dst = sw + lane * 36;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double lc = (double)lam[c];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        double w[W];
                        int ix[W];
                        load_axis<W>(wc, ic, ((long long)(3 * m + c) * 3 + a) * W, w, ix);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            double v = 0.0;
#pragma unroll
                            for (int q = 0; q < W; ++q) v += (ix[q] - org[a] == k) ? w[q] : 0.0;
                            dst[(c * 3 + a) * 4 + k] = (a == 2) ? v * lc : v;
                        }
                    }
                }
            }
            __syncthreads();
            for (int p = 0; p < cnt; ++p) {
                const double *w = sw + p * 36;
                acc0 += w[lx] * w[4 + ly] * w[8 + lz];
                acc1 += w[12 + lx] * w[16 + ly] * w[20 + lz];
                acc2 += w[24 + lx] * w[28 + ly] * w[32 + lz];
            }
            __syncthreads();
        }
        const int g0 = org[0] + lx, g1 = org[1] + ly, g2 = org[2] + lz;
        if (g0 < R.n[0] && g1 < R.n[1] && g2 < R.n[2]) {
            const long long lin = (long long)g0 + (long long)R.n[0] * ((long long)g1 + (long long)R.n[1] * g2);
            const long long o = levs ? levs[rep * RB_MAXLEV].off : R.off;
            const double sc = alpha / R.dV;
            if (!(R.bc[0] != RBFIB_PERIODIC && g0 == 0)) y[o + lin] += (TO)(sc * acc0);
            if (!(R.bc[1] != RBFIB_PERIODIC && g1 == 0)) y[o + R.N + lin] += (TO)(sc * acc1);
            if (!(R.bc[2] != RBFIB_PERIODIC && g2 == 0)) y[o + 2 * R.N + lin] += (TO)(sc * acc2);
        }
    }
}

template <typename TO, typename TL>
static void spread_into(Ctx &c, MarkerSet &ms, const TL *lam_state, TO *y, double alpha, const LevDev *levs) {
    if (c.nm == 0) return;
    // grid-stride over the tiles that have pairs, with the launch geometry's grid and
    // pairs per LDS round
    const int grid = std::min(c.ntiles, c.tune.spread_grid);
    const int P = c.tune.spread_p;
    auto kern = c.kw == 6 ? (P == 16 ? k_spread<TO, TL, 6, 16> : (P == 64 ? k_spread<TO, TL, 6, 64> : k_spread<TO, TL, 6, 32>))
                          : (P == 16 ? k_spread<TO, TL, 4, 16> : (P == 64 ? k_spread<TO, TL, 4, 64> : k_spread<TO, TL, 4, 32>));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, c.stream, c.d_reps, c.d_tile_rep, ms.active, ms.n_active,
                       ms.pair_start, ms.pair_count, ms.pair_cap, ms.pair_m, ms.wc, ms.ic, lam_state, y, alpha, c.mask,
                       levs);
}

// y_fluid += alpha * S lambda, lambda read from the lambda slots of lam_state.
template <typename TL>
void launch_spread(Ctx &c, MarkerSet &ms, const TL *lam_state, double *y, double alpha) {
    spread_into<double, TL>(c, ms, lam_state, y, alpha, nullptr);
}
template void launch_spread<double>(Ctx &, MarkerSet &, const double *, double *, double);
template void launch_spread<float>(Ctx &, MarkerSet &, const float *, double *, double);

// Level 0 of the multigrid pool (velocity components) += alpha * S lambda.
template <typename T, typename TL>
void launch_spread_level0(Ctx &c, MarkerSet &ms, const TL *lam_state, T *pool, double alpha) {
    spread_into<T, TL>(c, ms, lam_state, pool, alpha, c.d_levs);
}
template void launch_spread_level0<float, double>(Ctx &, MarkerSet &, const double *, float *, double);
template void launch_spread_level0<float, float>(Ctx &, MarkerSet &, const float *, float *, double);
template void launch_spread_level0<double, double>(Ctx &, MarkerSet &, const double *, double *, double);

// ------------------------------------------------------------------ J, K, K^T per body
// y_lambda = -J v + K U ;  y_U = K^T lambda  (rows 3 and 4 of the saddle operator).
template <typename TX, int W>
__global__ void k_body_apply(const RepDev *reps, const int *body_rep, const int *body_off, const double *r,
                             const double *d, const TX *__restrict__ x, double *__restrict__ y,
                             const int *__restrict__ mask, const double *__restrict__ wc, const int *__restrict__ ic) {
    extern __shared__ double sred[];   // [nmp][6]
    int p = blockIdx.x;
    if (mask && !mask[body_rep[p]]) return;
    const RepDev &R = reps[body_rep[p]];
    int m0 = body_off[p], m1 = body_off[p + 1], nmp = m1 - m0;
    long long lam0 = R.off + 4 * R.N;
    long long U0 = lam0 + 3LL * R.nm + 6LL * (p - R.b0);
    double U[6];
    for (int k = 0; k < 6; ++k) U[k] = (double)x[U0 + k];
    for (int task = threadIdx.x; task < 3 * nmp; task += blockDim.x) {
        int i = task / 3, c = task % 3, m = m0 + i;
        double Jv = interp_cached<W>(R, wc, ic, m, c, x + R.off + c * R.N);
        const double *dm = d + 3 * m;
        double wxd[3] = {U[4] * dm[2] - U[5] * dm[1], U[5] * dm[0] - U[3] * dm[2], U[3] * dm[1] - U[4] * dm[0]};
        y[lam0 + 3LL * (m - R.m0) + c] = -Jv + U[c] + wxd[c];
    }
    for (int i = threadIdx.x; i < nmp; i += blockDim.x) {
        int m = m0 + i;
        const TX *lx = x + lam0 + 3LL * (m - R.m0);
        const double l[3] = {(double)lx[0], (double)lx[1], (double)lx[2]};
        const double *dm = d + 3 * m;
        sred[6 * i + 0] = l[0];
        sred[6 * i + 1] = l[1];
        sred[6 * i + 2] = l[2];
        sred[6 * i + 3] = dm[1] * l[2] - dm[2] * l[1];
        sred[6 * i + 4] = dm[2] * l[0] - dm[0] * l[2];
        sred[6 * i + 5] = dm[0] * l[1] - dm[1] * l[0];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int i = 0; i < nmp; ++i) s += sred[6 * i + threadIdx.x];
        y[U0 + threadIdx.x] = s;
    }
}

template <typename TX>
void launch_body_apply(Ctx &c, MarkerSet &ms, const double *q, const TX *x, double *y) {
    (void)q;
    if (c.nb == 0) return;
    size_t sh = sizeof(double) * 6 * (size_t)c.max_body_nm;
    if (c.kw == 6)
        hipLaunchKernelGGL((k_body_apply<TX, 6>), dim3(c.nb), dim3(128), sh, c.stream, c.d_reps, c.d_body_rep,
                           c.d_body_off, ms.r, ms.d, x, y, c.mask, ms.wc, ms.ic);
    else
        hipLaunchKernelGGL((k_body_apply<TX, 4>), dim3(c.nb), dim3(128), sh, c.stream, c.d_reps, c.d_body_rep,
                           c.d_body_off, ms.r, ms.d, x, y, c.mask, ms.wc, ms.ic);
}
template void launch_body_apply<double>(Ctx &, MarkerSet &, const double *, const double *, double *);
template void launch_body_apply<float>(Ctx &, MarkerSet &, const double *, const float *, double *);

// ------------------------------------------------------------------ interpolation
// out[m, c] (= or +=) alpha * (J u)_c at markers of ms; u is a state vector.
template <int W>
__global__ void k_interp(const RepDev *reps, const int *marker_body, const int *body_rep, const double *wc,
                         const int *ic, int nm, const double *__restrict__ u, double *__restrict__ out, double alpha,
                         int accumulate) {
    int task = blockIdx.x * blockDim.x + threadIdx.x;
    if (task >= 3 * nm) return;
    int m = task / 3, c = task % 3;
    const RepDev &R = reps[body_rep[marker_body[m]]];
    double v = alpha * interp_cached<W>(R, wc, ic, m, c, u + R.off + c * R.N);
    if (accumulate) out[task] += v; else out[task] = v;
}

void launch_interp(Ctx &c, MarkerSet &ms, const double *u, double *out, double alpha, bool accumulate) {
    if (c.nm == 0) return;
    hipLaunchKernelGGL(c.kw == 6 ? k_interp<6> : k_interp<4>, dim3((3 * c.nm + 255) / 256), dim3(256), 0, c.stream,
                       c.d_reps, c.d_marker_body, c.d_body_rep, ms.wc, ms.ic, c.nm, u, out, alpha, accumulate ? 1 : 0);
}

// Affine part of interpolation next to sliding walls: for each support point across a
// wall moving with tangential velocity U (component c), add w * 2U * (product of the
// signs of the point's other reflections).  out[m, c] += alpha * J_bc.
template <int W>
__global__ void k_interp_bc(const RepDev *reps, const int *marker_body, const int *body_rep, const double *r, int nm,
                            double *__restrict__ out, double alpha) {
    int task = blockIdx.x * blockDim.x + threadIdx.x;
    if (task >= 3 * nm) return;
    int m = task / 3, c = task % 3;
    const RepDev &R = reps[body_rep[marker_body[m]]];
    if (!R.movwall) return;
    int idx[3][W], cr[3][W];
    double w[3][W];
    for (int a = 0; a < 3; ++a) axis_weights<W>(R, r[3 * m + a], c, a, idx[a], w[a], cr[a]);
    double acc = 0.0;
    for (int z = 0; z < W; ++z)
        for (int y = 0; y < W; ++y)
            for (int x = 0; x < W; ++x) {
                double wt = w[0][x] * w[1][y] * w[2][z];
                if (wt == 0.0) continue;
                int crs[3] = {cr[0][x], cr[1][y], cr[2][z]};
                // w carries the product of all reflection signs; divide out the one of
                // the moving wall itself (multiply by -1 again) to keep the others'.
                double aff = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (a == c || crs[a] == 0 || R.bc[a] != RBFIB_WALL) continue;
                    double U = R.wv[a][crs[a] - 1][c];
                    if (U != 0.0) aff += -2.0 * U;
                }
                acc += wt * aff;
            }
    out[task] += alpha * acc;
}

void launch_interp_bc(Ctx &c, MarkerSet &ms, double *out, double alpha) {
    if (c.nm == 0) return;
    hipLaunchKernelGGL(c.kw == 6 ? k_interp_bc<6> : k_interp_bc<4>, dim3((3 * c.nm + 255) / 256), dim3(256), 0,
                       c.stream, c.d_reps, c.d_marker_body, c.d_body_rep, ms.r, c.nm, out, alpha);
}

// ------------------------------------------------------------------ body block of P^-1
// Per body, in the body frame (rotation by R^T): U' = N (r_U' + K^T Minv g'),
// lambda' = Minv K U' - Minv g', with Minv the inverse blob mobility of the
// reference body; rotated back to the lab frame.
template <typename TZ>
__global__ void k_body_precond(const RepDev *reps, const int *body_rep, const int *body_off, const int *body_shape,
                               const ShapeDev *shapes, const double *sdata, const double *theta,
                               const double *__restrict__ rin, TZ *__restrict__ z,
                               const int *__restrict__ mask, const double *__restrict__ rs, int rstride) {
    extern __shared__ double sm[];
    int p = blockIdx.x;
    if (mask && !mask[body_rep[p]]) return;
    // rin is read as rin * f (f = rs[rep * rstride], 1 without rs)
    const double f = rs ? rs[(long long)body_rep[p] * rstride] : 1.0;
    const RepDev &R = reps[body_rep[p]];
    const ShapeDev &S = shapes[body_shape[p]];
    int m0 = body_off[p], n3 = 3 * S.nm;
    double *g = sm;            // [n3]
    double *a = sm + n3;       // [n3]
    double *b6 = sm + 2 * n3;  // [6]  body-frame rhs
    double *U6 = b6 + 6;       // [6]
    double Rm[9];
    quat_to_R(theta + 4 * p, Rm);
    long long lam0 = R.off + 4 * R.N + 3LL * (m0 - R.m0);
    long long U0 = R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0);
    for (int i = threadIdx.x; i < S.nm; i += blockDim.x) {
        const double *vi = rin + lam0 + 3 * i;
        const double v[3] = {vi[0] * f, vi[1] * f, vi[2] * f};
        for (int k = 0; k < 3; ++k) g[3 * i + k] = Rm[k] * v[0] + Rm[3 + k] * v[1] + Rm[6 + k] * v[2];
    }
    if (threadIdx.x < 2) {
        const double *vi = rin + U0 + 3 * threadIdx.x;
        const double v[3] = {vi[0] * f, vi[1] * f, vi[2] * f};
        for (int k = 0; k < 3; ++k) b6[3 * threadIdx.x + k] = Rm[k] * v[0] + Rm[3 + k] * v[1] + Rm[6 + k] * v[2];
    }
    __syncthreads();
    const double *Minv = sdata + S.minv_off;
    for (int k = threadIdx.x; k < n3; k += blockDim.x) {
        double s = 0.0;
        const double *row = Minv + (long long)k * n3;
        for (int j = 0; j < n3; ++j) s += row[j] * g[j];
        a[k] = s;
    }
    __syncthreads();
    const double *rr = sdata + S.rref_off;
    if (threadIdx.x < 6) {
        int k = threadIdx.x;
        double s = 0.0;
        for (int i = 0; i < S.nm; ++i) {
            const double *ai = a + 3 * i;
            const double *ri = rr + 3 * i;
            double v;
            if (k < 3) v = ai[k];
            else if (k == 3) v = ri[1] * ai[2] - ri[2] * ai[1];
            else if (k == 4) v = ri[2] * ai[0] - ri[0] * ai[2];
            else v = ri[0] * ai[1] - ri[1] * ai[0];
            s += v;
        }
        b6[k] += s;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const double *Nm = sdata + S.n_off;
        double s = 0.0;
        for (int l = 0; l < 6; ++l) s += Nm[6 * threadIdx.x + l] * b6[l];
        U6[threadIdx.x] = s;
    }
    __syncthreads();
    const double *MK = sdata + S.mk_off;
    for (int k = threadIdx.x; k < n3; k += blockDim.x) {
        double s = 0.0;
        for (int l = 0; l < 6; ++l) s += MK[6 * k + l] * U6[l];
        g[k] = s - a[k];       // lambda' (body frame), reuse g
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S.nm; i += blockDim.x) {
        const double *v = g + 3 * i;
        TZ *o = z + lam0 + 3 * i;
        for (int k = 0; k < 3; ++k) o[k] = (TZ)(Rm[3 * k] * v[0] + Rm[3 * k + 1] * v[1] + Rm[3 * k + 2] * v[2]);
    }
    if (threadIdx.x < 2) {
        const double *v = U6 + 3 * threadIdx.x;
        TZ *o = z + U0 + 3 * threadIdx.x;
        for (int k = 0; k < 3; ++k) o[k] = (TZ)(Rm[3 * k] * v[0] + Rm[3 * k + 1] * v[1] + Rm[3 * k + 2] * v[2]);
    }
}

template <typename TZ>
void launch_body_precond(Ctx &c, MarkerSet &ms, const double *theta, const double *r, TZ *z, const double *rs) {
    (void)ms;
    if (c.nb == 0) return;
    size_t sh = sizeof(double) * (size_t)(6 * c.max_body_nm + 12);
    hipLaunchKernelGGL(k_body_precond<TZ>, dim3(c.nb), dim3(128), sh, c.stream, c.d_reps, c.d_body_rep, c.d_body_off,
                       c.d_body_shape, c.d_shapes, c.d_shape_data, theta, r, z, c.mask, rs, c.m + 1);
}
template void launch_body_precond<double>(Ctx &, MarkerSet &, const double *, const double *, double *,
                                          const double *);
template void launch_body_precond<float>(Ctx &, MarkerSet &, const double *, const double *, float *,
                                         const double *);

// ------------------------------------------------------------------ small helpers
// zero the lambda and U slots of every replica
template <typename TY>
__global__ void k_zero_bodies(const RepDev *reps, int nrep, TY *y, const int *__restrict__ mask) {
    int r = blockIdx.y;
    if (r >= nrep || (mask && !mask[r])) return;
    const RepDev &R = reps[r];
    long long n = 3LL * R.nm + 6LL * R.nb;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        y[R.off + 4 * R.N + i] = (TY)0;
}

template <typename TY>
void launch_zero_bodies(Ctx &c, TY *y) {
    hipLaunchKernelGGL(k_zero_bodies<TY>, dim3(4, c.nrep), dim3(256), 0, c.stream, c.d_reps, c.nrep, y, c.mask);
}
template void launch_zero_bodies<double>(Ctx &, double *);
template void launch_zero_bodies<float>(Ctx &, float *);

// b = [0 ; 0 ; -slip ; FT]  (fluid rows zeroed; boundary terms added separately)
__global__ void k_set_rhs_bodies(const RepDev *reps, const int *marker_body, const int *body_rep, int nm, int nb,
                                 const double *FT, const double *slip, double *b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 3 * nm) {
        int m = t / 3, c = t % 3;
        const RepDev &R = reps[body_rep[marker_body[m]]];
        b[R.off + 4 * R.N + 3LL * (m - R.m0) + c] = slip ? -slip[t] : 0.0;
    }
    if (t < 6 * nb) {
        int p = t / 6, k = t % 6;
        const RepDev &R = reps[body_rep[p]];
        b[R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0) + k] = FT ? FT[t] : 0.0;
    }
}

void launch_set_rhs(Ctx &c, const double *FT, const double *slip, double *b) {
    int n = std::max(3 * c.nm, 6 * c.nb);
    if (n == 0) return;
    hipLaunchKernelGGL(k_set_rhs_bodies, dim3((n + 255) / 256), dim3(256), 0, c.stream, c.d_reps, c.d_marker_body,
                       c.d_body_rep, c.nm, c.nb, FT, slip, b);
}

// U[p] = scale * x_U[p]
__global__ void k_copy_U(const RepDev *reps, const int *body_rep, int nb, const double *x, double *U, double scale) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * nb) return;
    int p = t / 6, k = t % 6;
    const RepDev &R = reps[body_rep[p]];
    U[t] = scale * x[R.off + 4 * R.N + 3LL * R.nm + 6LL * (p - R.b0) + k];
}

void launch_copy_U(Ctx &c, const double *x, double *U, double scale) {
    if (c.nb == 0) return;
    hipLaunchKernelGGL(k_copy_U, dim3((6 * c.nb + 255) / 256), dim3(256), 0, c.stream, c.d_reps, c.d_body_rep, c.nb,
                       x, U, scale);
}

}  // namespace rb

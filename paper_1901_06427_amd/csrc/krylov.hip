// Flexible GMRES building blocks, batched over independent replicas.
// Every replica owns a contiguous segment of each state vector; blocks are
// replica-aligned chunks of RB_CHUNK elements, so per-replica dot products are
// block partial sums reduced in a fixed order (deterministic, no atomics).
// Hessenberg, Givens rotations and the least-squares solve live on the device,
// one thread per replica.
#include "common.h"

namespace rb {

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;   // valid in lane 0
}

// partial[blk * stride + i] = sum over the block's chunk of V_i . w.  The chunk of w
// is staged in LDS once; each wavefront then owns every fourth basis vector and
// reads its chunk of V_i with all sixteen loads per lane in flight together, so the
// vector loop needs no block barrier.  The basis streams through once per call:
// non-temporal loads keep it from displacing w and the partials in the caches
// (about 3 percent faster on the 256-replica ensemble; the basis update, which also
// writes w, is not helped by them).
__global__ __launch_bounds__(RB_BLOCK) void k_dot_partial(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                          long long L, int nvec, const double *__restrict__ w,
                                                          double *partial, int stride, const int *mask) {
    __shared__ double ws[RB_CHUNK];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    long long b = R.off + be.start;
    int n = (int)min((long long)RB_CHUNK, R.len - be.start);
    for (int k = threadIdx.x; k < RB_CHUNK; k += RB_BLOCK) ws[k] = (k < n) ? w[b + k] : 0.0;
    __syncthreads();
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < nvec; i += RB_BLOCK / 64) {
        const double *Vi = V + (long long)i * L + b;
        double v[RB_CHUNK / 64];
#pragma unroll
        for (int m = 0; m < RB_CHUNK / 64; ++m) {
            const int k = lane + 64 * m;
            v[m] = k < n ? __builtin_nontemporal_load(Vi + k) : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < RB_CHUNK / 64; ++m) acc = fma(v[m], ws[lane + 64 * m], acc);
        acc = wave_sum(acc);
        if (lane == 0) partial[(long long)blockIdx.x * stride + i] = acc;
    }
}

// out[r * out_stride + i] = sum of replica r's block partials of vector i, one
// wavefront per (replica, vector), fixed summation order; times scale[r * out_stride
// + i] when a scale is given.
// blockIdx.z = t selects the t-th of several sets: partial entries at + t * zin, outputs at
// + t * zout.
__global__ void k_dot_reduce(const int *first, const int *nblk, const double *partial, int stride, double *out,
                             int out_stride, const int *mask, int take_sqrt, const double *scale, int zin = 0,
                             long long zout = 0) {
    int r = blockIdx.x, i = blockIdx.y;
    if (mask && !mask[r]) return;
    const double *pp = partial + (long long)blockIdx.z * zin;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk[r]; b += 64) s += pp[(long long)(first[r] + b) * stride + i];
    s = wave_sum(s);
    if (scale) s *= scale[(long long)r * out_stride + i];
    if (threadIdx.x == 0) out[(long long)blockIdx.z * zout + (long long)r * out_stride + i] = take_sqrt ? sqrt(s) : s;
}

void launch_dots(Ctx &c, const double *V, int nvec, const double *w, double *out, const int *mask,
                 const double *scale) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(k_dot_partial, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, V,
                       c.L, nvec, w, c.partial, stride, mask);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, nvec), dim3(64), 0, c.stream, c.d_vec_first, c.d_vec_nblk,
                       c.partial, stride, out, c.m + 1, mask, 0, scale);
}

void launch_norm(Ctx &c, const double *w, double *out, const int *mask) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(k_dot_partial, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, w, c.L,
                       1, w, c.partial, stride, mask);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, 1), dim3(64), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
                       stride, out, 1, mask, 1, (const double *)nullptr);
}

// w += sign * sum_i coef[r][i] scale[r][i] V_i (scale 1 when not given); when
// partial is given, also the block partials of the updated w's squared norm.
__global__ __launch_bounds__(RB_BLOCK) void k_axpy_multi(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                         long long L, int nvec, const double *coef, int cstride,
                                                         const double *scale, double *__restrict__ w, double sign,
                                                         const int *mask, double *partial, int stride) {
    __shared__ double cf[RB_BLOCK];   // restart length <= 200 < RB_BLOCK
    __shared__ double red[RB_BLOCK / 64];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    if (threadIdx.x < nvec) {
        const long long ci = (long long)be.rep * cstride + threadIdx.x;
        cf[threadIdx.x] = sign * coef[ci] * (scale ? scale[ci] : 1.0);
    }
    __syncthreads();
    long long b = R.off + be.start;
    int n = (int)min((long long)RB_CHUNK, R.len - be.start);
    // four elements per thread; four basis vectors per step, so that sixteen loads
    // are in flight; each element sums its terms in increasing i
    constexpr int E = RB_CHUNK / RB_BLOCK;
    double acc[E];
    bool ok[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        acc[m] = 0.0;
        ok[m] = threadIdx.x + RB_BLOCK * m < n;
    }
    int i = 0;
    for (; i + 4 <= nvec; i += 4) {
        double v[4][E];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m)
                v[q][m] = ok[m] ? V[(long long)(i + q) * L + b + threadIdx.x + RB_BLOCK * m] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) acc[m] = fma(cf[i + q], v[q][m], acc[m]);
    }
    for (; i < nvec; ++i) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (ok[m]) acc[m] = fma(cf[i], V[(long long)i * L + b + threadIdx.x + RB_BLOCK * m], acc[m]);
    }
    double sq = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (!ok[m]) continue;
        const long long g = b + threadIdx.x + RB_BLOCK * m;
        const double v = w[g] + acc[m];
        w[g] = v;
        sq += v * v;
    }
    if (partial) {
        sq = wave_sum(sq);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sq;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int k = 0; k < RB_BLOCK / 64; ++k) s += red[k];
            partial[(long long)blockIdx.x * stride] = s;
        }
    }
}

void launch_axpy_multi(Ctx &c, const double *V, int nvec, const double *coef, double *w, double sign, const int *mask,
                       const double *scale) {
    hipLaunchKernelGGL(k_axpy_multi, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, V, c.L,
                       nvec, coef, c.m + 1, scale, w, sign, mask, (double *)nullptr, 0);
}

// w -= sum_i coef_i scale_i V_i and nrm[r] = ||w|| in two launches.
void launch_axpy_multi_norm(Ctx &c, const double *V, int nvec, const double *coef, double *w, double *nrm,
                            const int *mask, const double *scale) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(k_axpy_multi, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, V, c.L,
                       nvec, coef, c.m + 1, scale, w, -1.0, mask, c.partial, stride);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, 1), dim3(64), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
                       stride, nrm, 1, mask, 1, (const double *)nullptr);
}

// out = w * s[r]  (or w / s[r] when inverse; a zero divisor leaves out unchanged)
__global__ void k_scale(const RepDev *reps, const BlockEnt *tab, const double *w, const double *s, int sstride,
                        double *out, const int *mask, int inverse) {
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    double f = s[(long long)be.rep * sstride];
    if (inverse) {
        if (f == 0.0) return;
        f = 1.0 / f;
    }
    long long b = R.off + be.start;
    long long e = R.off + min(be.start + (long long)RB_CHUNK, R.len);
    for (long long g = b + threadIdx.x; g < e; g += RB_BLOCK) out[g] = w[g] * f;
}

void launch_scale(Ctx &c, const double *w, const double *s, double *out, const int *mask, bool inverse) {
    hipLaunchKernelGGL(k_scale, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, w, s, 1, out,
                       mask, inverse ? 1 : 0);
}

__global__ void k_axpby(const RepDev *reps, const BlockEnt *tab, double a, const double *x, double b,
                        const double *y, double *out, const int *mask) {
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    long long s = R.off + be.start;
    long long e = R.off + min(be.start + (long long)RB_CHUNK, R.len);
    for (long long g = s + threadIdx.x; g < e; g += RB_BLOCK) {
        double v = (a == 0.0 ? 0.0 : a * x[g]);
        if (b != 0.0) v += b * y[g];
        out[g] = v;
    }
}

void launch_axpby(Ctx &c, double a, const double *x, double b, const double *y, double *out, const int *mask) {
    hipLaunchKernelGGL(k_axpby, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, a, x, b, y,
                       out, mask);
}

void launch_copy(Ctx &c, const double *x, double *y, const int *mask) { launch_axpby(c, 1.0, x, 0.0, x, y, mask); }
void launch_zero(Ctx &c, double *y, const int *mask) { launch_axpby(c, 0.0, y, 0.0, y, y, mask); }

// Arnoldi column j: H[:, j] = h1 + h2 (two Gram-Schmidt passes), H[j+1, j] = ||w||;
// apply the stored rotations, form the new one, update g and the convergence state.
// New Hessenberg column k (entries e(i) for rows i <= k, hlast in row k+1): the earlier
// rotations 0..k-1 act on it in order, the entry each rotation passes on carried in a
// register (only the fused multiply-adds are serial), then rotation k is formed and
// applied to g.  Returns |g[k+1]|, the residual estimate, and den (row k of R).
template <class Entry>
__device__ __forceinline__ double givens_column(double *Hc, double *c, double *s, double *g, int k, Entry e,
                                                double hlast, double &den) {
    double x = e(0);
    for (int i = 0; i < k; ++i) {
        const double y = e(i + 1);
        Hc[i] = fma(c[i], x, s[i] * y);
        x = fma(-s[i], x, c[i] * y);
    }
    den = hypot(x, hlast);
    const double ck = den > 0.0 ? x / den : 1.0;
    const double sk = den > 0.0 ? hlast / den : 0.0;
    c[k] = ck;
    s[k] = sk;
    Hc[k] = den;
    Hc[k + 1] = 0.0;
    g[k + 1] = -sk * g[k];
    g[k] = ck * g[k];
    return fabs(g[k + 1]);
}

// The earlier rotations act on the new column h (= h1 + h2, then ||w||) in order; the
// entry each rotation passes on is carried in a register, so only its fused
// multiply-adds are serial (the loads of h, c and s are independent of them).
__global__ void k_givens(int nrep, int m, int j, double tol, const double *__restrict__ h1,
                         const double *__restrict__ h2, const double *__restrict__ nrm, double *__restrict__ H,
                         double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ gv,
                         const double *__restrict__ beta0, int *active, int *jf, int *status, int *iters,
                         double *__restrict__ inv_nu) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep || !active[r]) return;
    double *Hc = H + (long long)r * (m + 1) * m + (long long)j * (m + 1);
    double *c = cs + (long long)r * m, *s = sn + (long long)r * m, *g = gv + (long long)r * (m + 1);
    const double *a1 = h1 + (long long)r * (m + 1), *a2 = h2 + (long long)r * (m + 1);
    double hn = nrm[r];
    // basis vector j+1 is kept unnormalised: v_{j+1} = u_{j+1} / hn
    inv_nu[(long long)r * (m + 1) + j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    double den;
    const double res = givens_column(Hc, c, s, g, j, [&](int i) { return a1[i] + a2[i]; }, hn, den);
    iters[r] += 1;
    if (!isfinite(res) || !isfinite(den)) {
        status[r] = RBFIB_ENUMERIC;
        active[r] = 0;
        jf[r] = j;
        return;
    }
    if (res <= tol * beta0[r] || hn == 0.0) {
        active[r] = 0;
        jf[r] = j + 1;
        status[r] = RBFIB_OK;
    } else if (j + 1 == m) {
        jf[r] = m;
    }
}

void launch_givens(Ctx &c, int j, double tol) {
    double *h1 = c.hcol, *h2 = c.hcol + (long long)c.nrep * (c.m + 1), *nrm = c.hcol + 2LL * c.nrep * (c.m + 1);
    hipLaunchKernelGGL(k_givens, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.m, j, tol, h1, h2, nrm,
                       c.H, c.cs, c.sn, c.gv, c.beta0, c.active, c.jf, c.status, c.iters, c.inv_nu);
}

// ------------------------------------------------------------------ two-step blocks
// A block of two Arnoldi steps forms u_1 = A P^-1 v_j and u_2 = A P^-1 u_1 first, then
// orthogonalises both against v_0 .. v_j in one pass over the basis for the projections
// and one for the update, and against each other by a 2 x 2 Cholesky QR of their Gram
// matrix.  With z_j = P^-1 v_j and z_{j+1} = P^-1 u_1, A Z = V H holds with the
// projection coefficients and the Cholesky factors as the two new Hessenberg columns.

// partial[blk * stride + t * half + i] = the block's part of V_i . w_t (t = 0, 1)
__global__ __launch_bounds__(RB_BLOCK) void k_dot_partial2(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                           long long L, int nvec, const double *__restrict__ w1,
                                                           const double *__restrict__ w2, double *partial, int stride,
                                                           int half, const int *mask) {
    __shared__ double ws1[RB_CHUNK], ws2[RB_CHUNK];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    long long b = R.off + be.start;
    int n = (int)min((long long)RB_CHUNK, R.len - be.start);
    for (int k = threadIdx.x; k < RB_CHUNK; k += RB_BLOCK) {
        ws1[k] = (k < n) ? w1[b + k] : 0.0;
        ws2[k] = (k < n) ? w2[b + k] : 0.0;
    }
    __syncthreads();
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < nvec; i += RB_BLOCK / 64) {
        const double *Vi = V + (long long)i * L + b;
        double v[RB_CHUNK / 64];
#pragma unroll
        for (int m = 0; m < RB_CHUNK / 64; ++m) {
            const int k = lane + 64 * m;
            v[m] = k < n ? __builtin_nontemporal_load(Vi + k) : 0.0;
        }
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int m = 0; m < RB_CHUNK / 64; ++m) {
            a1 = fma(v[m], ws1[lane + 64 * m], a1);
            a2 = fma(v[m], ws2[lane + 64 * m], a2);
        }
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
            partial[(long long)blockIdx.x * stride + i] = a1;
            partial[(long long)blockIdx.x * stride + half + i] = a2;
        }
    }
}

// out1 / out2 [r][i] = scale[r][i] * (V_i . w1 / w2), out2 = out1 + nrep * (m + 1)
void launch_dots2(Ctx &c, const double *V, int nvec, const double *w1, const double *w2, double *out1,
                  const int *mask, const double *scale) {
    const int half = c.m + 1, stride = 2 * half;
    hipLaunchKernelGGL(k_dot_partial2, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, V,
                       c.L, nvec, w1, w2, c.partial, stride, half, mask);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, nvec, 2), dim3(64), 0, c.stream, c.d_vec_first, c.d_vec_nblk,
                       c.partial, stride, out1, c.m + 1, mask, 0, scale, half, (long long)c.nrep * (c.m + 1));
}

// u_t -= sum_i coef_t[r][i] scale[r][i] V_i (t = 1, 2), and the block partials of
// (u_1.u_1, u_1.u_2, u_2.u_2) after the update at partial[blk * stride + 0..2]
__global__ __launch_bounds__(RB_BLOCK) void k_axpy_multi2(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                          long long L, int nvec, const double *coef1,
                                                          const double *coef2, int cstride, const double *scale,
                                                          double *__restrict__ u1, double *__restrict__ u2,
                                                          const int *mask, double *partial, int stride) {
    __shared__ double cf1[RB_BLOCK], cf2[RB_BLOCK];   // restart length <= 200 < RB_BLOCK
    __shared__ double red[3][RB_BLOCK / 64];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    if (threadIdx.x < nvec) {
        const long long ci = (long long)be.rep * cstride + threadIdx.x;
        const double sc = scale ? scale[ci] : 1.0;
        cf1[threadIdx.x] = -coef1[ci] * sc;
        cf2[threadIdx.x] = -coef2[ci] * sc;
    }
    __syncthreads();
    long long b = R.off + be.start;
    int n = (int)min((long long)RB_CHUNK, R.len - be.start);
    constexpr int E = RB_CHUNK / RB_BLOCK;
    double a1[E], a2[E];
    bool ok[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        a1[m] = 0.0;
        a2[m] = 0.0;
        ok[m] = threadIdx.x + RB_BLOCK * m < n;
    }
    int i = 0;
    for (; i + 4 <= nvec; i += 4) {
        double v[4][E];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m)
                v[q][m] = ok[m] ? V[(long long)(i + q) * L + b + threadIdx.x + RB_BLOCK * m] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                a1[m] = fma(cf1[i + q], v[q][m], a1[m]);
                a2[m] = fma(cf2[i + q], v[q][m], a2[m]);
            }
    }
    for (; i < nvec; ++i) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (ok[m]) {
                const double vv = V[(long long)i * L + b + threadIdx.x + RB_BLOCK * m];
                a1[m] = fma(cf1[i], vv, a1[m]);
                a2[m] = fma(cf2[i], vv, a2[m]);
            }
    }
    double s11 = 0.0, s12 = 0.0, s22 = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (!ok[m]) continue;
        const long long g = b + threadIdx.x + RB_BLOCK * m;
        const double x1 = u1[g] + a1[m], x2 = u2[g] + a2[m];
        u1[g] = x1;
        u2[g] = x2;
        s11 = fma(x1, x1, s11);
        s12 = fma(x1, x2, s12);
        s22 = fma(x2, x2, s22);
    }
    s11 = wave_sum(s11);
    s12 = wave_sum(s12);
    s22 = wave_sum(s22);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s11;
        red[1][threadIdx.x >> 6] = s12;
        red[2][threadIdx.x >> 6] = s22;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double t = 0.0;
        for (int k = 0; k < RB_BLOCK / 64; ++k) t += red[threadIdx.x][k];
        partial[(long long)blockIdx.x * stride + threadIdx.x] = t;
    }
}

// gram[r][0..2] = (u_1.u_1, u_1.u_2, u_2.u_2) after the update
void launch_axpy2_gram(Ctx &c, const double *V, int nvec, const double *coef1, const double *coef2, double *u1,
                       double *u2, double *gram, const int *mask, const double *scale) {
    const int stride = 2 * (c.m + 1);
    hipLaunchKernelGGL(k_axpy_multi2, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, V, c.L,
                       nvec, coef1, coef2, c.m + 1, scale, u1, u2, mask, c.partial, stride);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, 3), dim3(64), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
                       stride, gram, 3, mask, 0, (const double *)nullptr, 0, 0LL);
}

// Columns j and j+1: R = chol(Gram) gives v_{j+1} = u_1 / r11 and, after the combine
// pass, v_{j+2} = (u_2 - (r12 / r11) u_1) / r22; column j holds the projections of u_1
// and r11, column j+1 those of u_2, r12 and r22.  A replica that converges at column j
// leaves column j+1 unused.
__global__ void k_givens2(int nrep, int m, int j, double tol, const double *__restrict__ h1,
                          const double *__restrict__ h2, const double *__restrict__ gram, double *__restrict__ H,
                          double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ gv,
                          const double *__restrict__ beta0, int *active, int *jf, int *status, int *iters,
                          double *__restrict__ inv_nu, double *__restrict__ tco) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep || !active[r]) return;
    const double *a1 = h1 + (long long)r * (m + 1), *a2 = h2 + (long long)r * (m + 1);
    const double g11 = gram[3 * r], g12 = gram[3 * r + 1], g22 = gram[3 * r + 2];
    const double r11 = sqrt(g11);
    const double r12 = r11 > 0.0 ? g12 / r11 : 0.0;
    const double d22 = g22 - r12 * r12;
    const double r22 = d22 > 0.0 ? sqrt(d22) : 0.0;
    double *nu = inv_nu + (long long)r * (m + 1);
    nu[j + 1] = r11 > 0.0 ? 1.0 / r11 : 0.0;
    nu[j + 2] = r22 > 0.0 ? 1.0 / r22 : 0.0;
    tco[r] = r11 > 0.0 ? r12 / r11 : 0.0;
    double *c = cs + (long long)r * m, *s = sn + (long long)r * m, *g = gv + (long long)r * (m + 1);
    double *H0 = H + (long long)r * (m + 1) * m + (long long)j * (m + 1);
    double den;
    double res = givens_column(H0, c, s, g, j, [&](int i) { return a1[i]; }, r11, den);
    iters[r] += 1;
    if (!isfinite(res) || !isfinite(den)) {
        status[r] = RBFIB_ENUMERIC;
        active[r] = 0;
        jf[r] = j;
        return;
    }
    if (res <= tol * beta0[r] || r11 == 0.0) {
        active[r] = 0;
        jf[r] = j + 1;
        status[r] = RBFIB_OK;
        return;
    }
    res = givens_column(H0 + (m + 1), c, s, g, j + 1, [&](int i) { return i <= j ? a2[i] : r12; }, r22, den);
    iters[r] += 1;
    if (!isfinite(res) || !isfinite(den)) {
        status[r] = RBFIB_ENUMERIC;
        active[r] = 0;
        jf[r] = j + 1;
        return;
    }
    if (res <= tol * beta0[r] || r22 == 0.0) {
        active[r] = 0;
        jf[r] = j + 2;
        status[r] = RBFIB_OK;
    } else if (j + 2 == m) {
        jf[r] = m;
    }
}

void launch_givens2(Ctx &c, int j, double tol) {
    double *h1 = c.hcol, *h2 = c.hcol + (long long)c.nrep * (c.m + 1);
    hipLaunchKernelGGL(k_givens2, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.m, j, tol, h1, h2,
                       c.gram, c.H, c.cs, c.sn, c.gv, c.beta0, c.active, c.jf, c.status, c.iters, c.inv_nu, c.tco);
}

// u_2 -= tco[r] u_1 (replicas still active)
__global__ void k_combine(const RepDev *reps, const BlockEnt *tab, const double *__restrict__ u1,
                          double *__restrict__ u2, const double *__restrict__ tco, const int *mask) {
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    const double f = tco[be.rep];
    long long b = R.off + be.start;
    long long e = R.off + min(be.start + (long long)RB_CHUNK, R.len);
    for (long long g = b + threadIdx.x; g < e; g += RB_BLOCK) u2[g] = fma(-f, u1[g], u2[g]);
}

void launch_combine(Ctx &c, const double *u1, double *u2, const int *mask) {
    hipLaunchKernelGGL(k_combine, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, u1, u2,
                       c.tco, mask);
}

// Back substitution H[0:jf, 0:jf] y = g[0:jf] for replicas active at cycle start.
__global__ void k_trisolve(int nrep, int m, const double *H, const double *gv, const int *cyc, const int *jf,
                           double *y) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep || !cyc[r]) return;
    int n = jf[r];
    const double *Hr = H + (long long)r * (m + 1) * m;
    const double *g = gv + (long long)r * (m + 1);
    double *yr = y + (long long)r * (m + 1);
    for (int i = n - 1; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k < n; ++k) s -= Hr[(long long)k * (m + 1) + i] * yr[k];
        double d = Hr[(long long)i * (m + 1) + i];
        yr[i] = d != 0.0 ? s / d : 0.0;
    }
    for (int i = n; i < m; ++i) yr[i] = 0.0;
}

// x += sum_{i < jf} y_i Z_i
// (the column loop is unrolled so that eight loads, one basis vector apart, are in
// flight together; the sum keeps its order)
__global__ __launch_bounds__(RB_BLOCK) void k_update_x(const RepDev *reps, const BlockEnt *tab,
                                                       const double *__restrict__ Z, long long L, int m,
                                                       const double *__restrict__ y, const int *jf, const int *cyc,
                                                       double *__restrict__ x) {
    BlockEnt be = tab[blockIdx.x];
    if (!cyc[be.rep]) return;
    const RepDev &R = reps[be.rep];
    int n = jf[be.rep];
    const double *yr = y + (long long)be.rep * (m + 1);
    long long b = R.off + be.start;
    long long e = R.off + min(be.start + (long long)RB_CHUNK, R.len);
    for (long long g = b + threadIdx.x; g < e; g += RB_BLOCK) {
        double acc = 0.0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) acc += yr[i] * Z[(long long)i * L + g];
        x[g] += acc;
    }
}

void launch_trisolve_update(Ctx &c) {
    hipLaunchKernelGGL(k_trisolve, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.m, c.H, c.gv,
                       c.cyc_active, c.jf, c.yv);
    hipLaunchKernelGGL(k_update_x, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, c.Z, c.L,
                       c.m, c.yv, c.jf, c.cyc_active, c.xsol);
}

// Start of a restart cycle for active replicas: g = (beta, 0, ...), jf = 0; beta in nrm slot.
__global__ void k_start_cycle(int nrep, int m, const double *beta, double *gv, int *active, int *jf, int *cyc,
                              int *status, double *inv_nu) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    cyc[r] = active[r];
    if (!active[r]) return;
    inv_nu[(long long)r * (m + 1)] = 1.0;   // the cycle's first basis vector is stored normalised
    double *g = gv + (long long)r * (m + 1);
    g[0] = beta[r];
    for (int i = 1; i <= m; ++i) g[i] = 0.0;
    jf[r] = 0;
    if (!isfinite(beta[r])) { status[r] = RBFIB_ENUMERIC; active[r] = 0; cyc[r] = 0; }
}

void launch_start_cycle(Ctx &c) {
    double *nrm = c.hcol + 2LL * c.nrep * (c.m + 1);
    hipLaunchKernelGGL(k_start_cycle, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.m, nrm, c.gv,
                       c.active, c.jf, c.cyc_active, c.status, c.inv_nu);
}

}  // namespace rb

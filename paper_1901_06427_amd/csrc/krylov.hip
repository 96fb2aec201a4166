// Flexible GMRES building blocks, batched over independent replicas.
// Every replica owns a contiguous segment of each state vector; blocks are
// replica-aligned chunks of CH elements (512, 1024 or 2048, the context's launch
// geometry; the vector block table carries CH / RB_BLOCK as its points per thread),
// so per-replica dot products are block partial sums reduced in a fixed order
// (deterministic, no atomics).
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
template <int CH>
__global__ __launch_bounds__(RB_BLOCK) void k_dot_partial(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                          long long L, int nvec, const double *__restrict__ w,
                                                          double *partial, int stride, const int *mask) {
    __shared__ double ws[CH];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    long long b = R.off + be.start;
    int n = (int)min((long long)CH, R.len - be.start);
    for (int k = threadIdx.x; k < CH; k += RB_BLOCK) ws[k] = (k < n) ? w[b + k] : 0.0;
    __syncthreads();
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < nvec; i += RB_BLOCK / 64) {
        const double *Vi = V + (long long)i * L + b;
        double v[CH / 64];
#pragma unroll
        for (int m = 0; m < CH / 64; ++m) {
            const int k = lane + 64 * m;
            v[m] = k < n ? __builtin_nontemporal_load(Vi + k) : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < CH / 64; ++m) acc = fma(v[m], ws[lane + 64 * m], acc);
        acc = wave_sum(acc);
        if (lane == 0) partial[(long long)blockIdx.x * stride + i] = acc;
    }
}

// out[r * out_stride + i] = sum of replica r's block partials of vector i, one
// wavefront per (replica, vector), fixed summation order; times scale[r * out_stride
// + i] when a scale is given.
// blockIdx.z = t selects the t-th of several sets: partial entries at + t * zin, outputs at
// + t * zout.
#define RB_RED 256   // threads of the partial-sum reduction
__global__ __launch_bounds__(RB_RED) void k_dot_reduce(const int *first, const int *nblk, const double *partial, int stride, double *out,
                             int out_stride, const int *mask, int take_sqrt, const double *scale, int zin = 0,
                             long long zout = 0) {
    int r = blockIdx.x, i = blockIdx.y;
    if (mask && !mask[r]) return;
    const double *pp = partial + (long long)blockIdx.z * zin + (long long)first[r] * stride + i;
    // RB_RED threads, four independent sums each (a single large replica has
    // thousands of block partials per vector), then the workgroup's waves combined
    const int n = nblk[r];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * RB_RED < n; b += 4 * RB_RED) {
        s0 += pp[(long long)b * stride];
        s1 += pp[(long long)(b + RB_RED) * stride];
        s2 += pp[(long long)(b + 2 * RB_RED) * stride];
        s3 += pp[(long long)(b + 3 * RB_RED) * stride];
    }
    for (; b < n; b += RB_RED) s0 += pp[(long long)b * stride];
    double s = wave_sum((s0 + s1) + (s2 + s3));
    __shared__ double red[RB_RED / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        s = red[0];
        for (int k = 1; k < RB_RED / 64; ++k) s += red[k];
        if (scale) s *= scale[(long long)r * out_stride + i];
        out[(long long)blockIdx.z * zout + (long long)r * out_stride + i] = take_sqrt ? sqrt(s) : s;
    }
}

// the kernel instance of the context's Krylov chunk
#define RB_BY_CHUNK(c, K, ...) \
    ((c).tune.krylov_chunk == 512 ? K<__VA_ARGS__ 512> : ((c).tune.krylov_chunk == 2048 ? K<__VA_ARGS__ 2048> : K<__VA_ARGS__ 1024>))

void launch_dots(Ctx &c, const double *V, int nvec, const double *w, double *out, const int *mask,
                 const double *scale) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_dot_partial, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_tab_vec, V, c.L, nvec, w, c.partial, stride, mask);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, nvec), dim3(RB_RED), 0, c.stream, c.d_vec_first, c.d_vec_nblk,
                       c.partial, stride, out, c.m + 1, mask, 0, scale);
}

void launch_norm(Ctx &c, const double *w, double *out, const int *mask) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_dot_partial, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_tab_vec, w, c.L, 1, w, c.partial, stride, mask);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, 1), dim3(RB_RED), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
                       stride, out, 1, mask, 1, (const double *)nullptr);
}

// w += sign * sum_i coef[r][i] scale[r][i] V_i (scale 1 when not given); when
// partial is given, also the block partials of the updated w's squared norm.
template <int CH>
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
    int n = (int)min((long long)CH, R.len - be.start);
    // CH / RB_BLOCK elements per thread; four basis vectors per step, so that four
    // loads per element are in flight; each element sums its terms in increasing i
    constexpr int E = CH / RB_BLOCK;
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
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_axpy_multi, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_tab_vec, V, c.L, nvec, coef, c.m + 1, scale, w, sign, mask, (double *)nullptr, 0);
}

// w -= sum_i coef_i scale_i V_i and nrm[r] = ||w|| in two launches.
void launch_axpy_multi_norm(Ctx &c, const double *V, int nvec, const double *coef, double *w, double *nrm,
                            const int *mask, const double *scale) {
    int stride = c.m + 1;
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_axpy_multi, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                       c.d_tab_vec, V, c.L, nvec, coef, c.m + 1, scale, w, -1.0, mask, c.partial, stride);
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, 1), dim3(RB_RED), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
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
    long long e = R.off + min(be.start + (long long)be.npt * RB_BLOCK, R.len);
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
    long long e = R.off + min(be.start + (long long)be.npt * RB_BLOCK, R.len);
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

// ------------------------------------------------------------------ s-step blocks
// A block of S Arnoldi steps (S = 2..4) forms u_1 = A P^-1 v_j and u_{k+1} = A P^-1 u_k
// first (in basis slots j+1 .. j+S), then orthogonalises all S against v_0 .. v_j with
// one projection pass and one update pass over the basis, and among themselves by a
// Cholesky QR of their S x S Gram matrix (accumulated by the update pass).  With
// z_j = P^-1 v_j and z_{j+k} = P^-1 u_k, A Z = V H holds with the projection
// coefficients and the Cholesky factor R as the S new Hessenberg columns, so flexible
// GMRES applies unchanged.  The basis is streamed once per S steps.

// partial[blk * stride + t * half + i] = the block's part of V_i . w_t, w_t = W + t L
template <int S, int CH>
__global__ __launch_bounds__(RB_BLOCK) void k_dot_partial_s(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                            long long L, int nvec, const double *W, double *partial,
                                                            int stride, int half, const int *mask) {
    __shared__ double ws[S][CH];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    long long b = R.off + be.start;
    int n = (int)min((long long)CH, R.len - be.start);
    for (int k = threadIdx.x; k < CH; k += RB_BLOCK)
#pragma unroll
        for (int t = 0; t < S; ++t) ws[t][k] = (k < n) ? W[(long long)t * L + b + k] : 0.0;
    __syncthreads();
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = wid; i < nvec; i += RB_BLOCK / 64) {
        const double *Vi = V + (long long)i * L + b;
        double v[CH / 64];
#pragma unroll
        for (int m = 0; m < CH / 64; ++m) {
            const int k = lane + 64 * m;
            v[m] = k < n ? __builtin_nontemporal_load(Vi + k) : 0.0;
        }
        double a[S];
#pragma unroll
        for (int t = 0; t < S; ++t) a[t] = 0.0;
#pragma unroll
        for (int m = 0; m < CH / 64; ++m)
#pragma unroll
            for (int t = 0; t < S; ++t) a[t] = fma(v[m], ws[t][lane + 64 * m], a[t]);
#pragma unroll
        for (int t = 0; t < S; ++t) {
            const double st = wave_sum(a[t]);
            if (lane == 0) partial[(long long)blockIdx.x * stride + t * half + i] = st;
        }
    }
}

// u_t -= sum_i coef[t][r][i] scale[r][i] V_i (t < S, u_t = W + t L, coef sets nrep (m+1)
// apart), and the block partials of the upper triangle of the Gram matrix of the
// updated u (row-major, S (S + 1) / 2 entries) at partial[blk * stride + q]
template <int S, int CH>
__global__ __launch_bounds__(RB_BLOCK) void k_axpy_multi_s(const RepDev *reps, const BlockEnt *tab, const double *V,
                                                           long long L, int nvec, const double *coef,
                                                           long long cset, int cstride, const double *scale,
                                                           double *W, const int *mask, double *partial, int stride) {
    constexpr int NG = S * (S + 1) / 2;
    __shared__ double cf[S][RB_BLOCK];   // restart length <= 200 < RB_BLOCK
    __shared__ double red[NG][RB_BLOCK / 64];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    if (threadIdx.x < nvec) {
        const long long ci = (long long)be.rep * cstride + threadIdx.x;
        const double sc = scale ? scale[ci] : 1.0;
#pragma unroll
        for (int t = 0; t < S; ++t) cf[t][threadIdx.x] = -coef[t * cset + ci] * sc;
    }
    __syncthreads();
    long long b = R.off + be.start;
    int n = (int)min((long long)CH, R.len - be.start);
    constexpr int E = CH / RB_BLOCK;
    double a[S][E];
    bool ok[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        ok[m] = threadIdx.x + RB_BLOCK * m < n;
#pragma unroll
        for (int t = 0; t < S; ++t) a[t][m] = 0.0;
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
            for (int m = 0; m < E; ++m)
#pragma unroll
                for (int t = 0; t < S; ++t) a[t][m] = fma(cf[t][i + q], v[q][m], a[t][m]);
    }
    for (; i < nvec; ++i) {
#pragma unroll
        for (int m = 0; m < E; ++m)
            if (ok[m]) {
                const double vv = V[(long long)i * L + b + threadIdx.x + RB_BLOCK * m];
#pragma unroll
                for (int t = 0; t < S; ++t) a[t][m] = fma(cf[t][i], vv, a[t][m]);
            }
    }
    double gs[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) gs[q] = 0.0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
        if (!ok[m]) continue;
        const long long g = b + threadIdx.x + RB_BLOCK * m;
        double x[S];
#pragma unroll
        for (int t = 0; t < S; ++t) {
            x[t] = W[(long long)t * L + g] + a[t][m];
            W[(long long)t * L + g] = x[t];
        }
        int q = 0;
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
            for (int t = p; t < S; ++t) gs[q] = fma(x[p], x[t], gs[q]), ++q;
    }
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const double w = wave_sum(gs[q]);
        if ((threadIdx.x & 63) == 0) red[q][threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x < NG) {
        double t = 0.0;
        for (int k = 0; k < RB_BLOCK / 64; ++k) t += red[threadIdx.x][k];
        partial[(long long)blockIdx.x * stride + threadIdx.x] = t;
    }
}

// hblk[t][r][i] = scale[r][i] (V_i . u_t), u_t = W + t L
void launch_block_dots(Ctx &c, int S, const double *V, int nvec, const double *W, const int *mask,
                       const double *scale) {
    const int half = c.m + 1, stride = RB_MAXS * half;
    const long long cset = (long long)c.nrep * (c.m + 1);
#define RB_DOTS(SS)                                                                                                  \
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_dot_partial_s, SS, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, \
                       c.d_tab_vec, V, c.L, nvec, W, c.partial, stride, half, mask)
    if (S == 2) RB_DOTS(2);
    else if (S == 3) RB_DOTS(3);
    else RB_DOTS(4);
#undef RB_DOTS
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, nvec, S), dim3(RB_RED), 0, c.stream, c.d_vec_first, c.d_vec_nblk,
                       c.partial, stride, c.hblk, c.m + 1, mask, 0, scale, half, cset);
}

// u_t -= sum_i hblk[t][r][i] scale[r][i] V_i; gram[r][q] = upper triangle of U^T U after it
void launch_block_update(Ctx &c, int S, const double *V, int nvec, double *W, const int *mask, const double *scale) {
    const int stride = RB_MAXS * (c.m + 1);
    const long long cset = (long long)c.nrep * (c.m + 1);
#define RB_UPD(SS)                                                                                                   \
    hipLaunchKernelGGL(RB_BY_CHUNK(c, k_axpy_multi_s, SS, ), dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, \
                       c.d_tab_vec, V, c.L, nvec, c.hblk, cset, c.m + 1, scale, W, mask, c.partial, stride)
    if (S == 2) RB_UPD(2);
    else if (S == 3) RB_UPD(3);
    else RB_UPD(4);
#undef RB_UPD
    const int ng = S * (S + 1) / 2;
    hipLaunchKernelGGL(k_dot_reduce, dim3(c.nrep, ng), dim3(RB_RED), 0, c.stream, c.d_vec_first, c.d_vec_nblk, c.partial,
                       stride, c.gram, RB_MAXG, mask, 0, (const double *)nullptr, 0, 0LL);
}

// Columns j .. j+S-1: the Cholesky factor R of the Gram matrix gives v_{j+k} = w_k / R_kk
// with w_1 = u_1, w_k = u_k - sum_{l<k} (R_lk / R_ll) w_l (the combine pass);
// column j+k-1 holds the projections of u_k and R_1k .. R_kk.  A replica that
// converges (or whose Gram matrix loses rank) at a column leaves the later ones unused.
template <int S>
__global__ void k_givens_s(int nrep, int m, int j, double tol, const double *__restrict__ hblk,
                           const double *__restrict__ gram, double *__restrict__ H, double *__restrict__ cs,
                           double *__restrict__ sn, double *__restrict__ gv, const double *__restrict__ beta0,
                           int *active, int *jf, int *status, int *iters, double *__restrict__ inv_nu,
                           double *__restrict__ tco) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep || !active[r]) return;
    const long long cset = (long long)nrep * (m + 1);
    // Cholesky factor of the packed upper triangle (all loops unrolled: constant indices)
    const double *gr = gram + (long long)r * RB_MAXG;
    double G[S][S], Rm[S][S];
    {
        int q = 0;
#pragma unroll
        for (int p = 0; p < S; ++p)
#pragma unroll
            for (int t = 0; t < S; ++t) {
                Rm[p][t] = 0.0;
                if (t >= p) G[p][t] = gr[q++];
                else G[p][t] = 0.0;
            }
    }
    int rank = S;   // leading columns with a positive pivot
#pragma unroll
    for (int t = 0; t < S; ++t) {
        double d = G[t][t];
#pragma unroll
        for (int p = 0; p < t; ++p) d -= Rm[p][t] * Rm[p][t];
        const bool ok = rank == S && d > 0.0;
        if (!ok && rank == S) rank = t;
        Rm[t][t] = ok ? sqrt(d) : 0.0;
#pragma unroll
        for (int u = t + 1; u < S; ++u) {
            double e = G[t][u];
#pragma unroll
            for (int p = 0; p < t; ++p) e -= Rm[p][t] * Rm[p][u];
            Rm[t][u] = ok ? e / Rm[t][t] : 0.0;
        }
    }
    double *nu = inv_nu + (long long)r * (m + 1);
    double *T = tco + (long long)r * RB_MAXS * RB_MAXS;
#pragma unroll
    for (int k = 0; k < S; ++k) nu[j + 1 + k] = Rm[k][k] > 0.0 ? 1.0 / Rm[k][k] : 0.0;
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
        for (int k = 0; k < S; ++k) T[l * RB_MAXS + k] = (l < k && Rm[l][l] > 0.0) ? Rm[l][k] / Rm[l][l] : 0.0;
    double *c = cs + (long long)r * m, *s = sn + (long long)r * m, *g = gv + (long long)r * (m + 1);
    double *H0 = H + (long long)r * (m + 1) * m + (long long)j * (m + 1);
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double *a = hblk + k * cset + (long long)r * (m + 1);
        // column j+k: rows 0..j the projections of u_{k+1}, rows j+1 .. j+k+1 R[0..k][k]
        double rc[S];
#pragma unroll
        for (int p = 0; p < S; ++p) rc[p] = Rm[p][k];
        auto entry = [&](int i) {
            if (i <= j) return a[i];
            const int d = i - j - 1;
            double v = 0.0;
#pragma unroll
            for (int p = 0; p < S; ++p) v = (d == p) ? rc[p] : v;
            return v;
        };
        const double last = rc[k];
        double den;
        const double res = givens_column(H0 + (long long)k * (m + 1), c, s, g, j + k, entry, last, den);
        iters[r] += 1;
        if (!isfinite(res) || !isfinite(den)) {
            status[r] = RBFIB_ENUMERIC;
            active[r] = 0;
            jf[r] = j + k;
            return;
        }
        if (res <= tol * beta0[r] || !(last > 0.0)) {
            active[r] = 0;
            jf[r] = j + k + 1;
            status[r] = RBFIB_OK;
            return;
        }
    }
    (void)rank;
    if (j + S == m) jf[r] = m;
}

void launch_givens_s(Ctx &c, int j, int S, double tol) {
#define RB_GIV(SS)                                                                                                   \
    hipLaunchKernelGGL(k_givens_s<SS>, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.m, j, tol, c.hblk, \
                       c.gram, c.H, c.cs, c.sn, c.gv, c.beta0, c.active, c.jf, c.status, c.iters, c.inv_nu, c.tco)
    if (S == 2) RB_GIV(2);
    else if (S == 3) RB_GIV(3);
    else RB_GIV(4);
#undef RB_GIV
}

// w_1 = u_1, w_k = u_k - sum_{l<k} T[l][k] w_l in place (slots W + t L), active replicas
template <int S>
__global__ void k_combine_s(const RepDev *reps, const BlockEnt *tab, long long L, double *W,
                            const double *__restrict__ tco, const int *mask) {
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const RepDev &R = reps[be.rep];
    const double *T = tco + (long long)be.rep * RB_MAXS * RB_MAXS;
    double f[S][S];
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
        for (int k = 0; k < S; ++k) f[l][k] = T[l * RB_MAXS + k];
    long long b = R.off + be.start;
    long long e = R.off + min(be.start + (long long)be.npt * RB_BLOCK, R.len);
    for (long long g = b + threadIdx.x; g < e; g += RB_BLOCK) {
        double w[S];
#pragma unroll
        for (int k = 0; k < S; ++k) w[k] = W[(long long)k * L + g];
#pragma unroll
        for (int k = 1; k < S; ++k) {
#pragma unroll
            for (int l = 0; l < k; ++l) w[k] = fma(-f[l][k], w[l], w[k]);
            W[(long long)k * L + g] = w[k];
        }
    }
}

void launch_combine_s(Ctx &c, int S, double *W, const int *mask) {
#define RB_CMB(SS)                                                                                                   \
    hipLaunchKernelGGL(k_combine_s<SS>, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec, c.L, W, \
                       c.tco, mask)
    if (S == 2) RB_CMB(2);
    else if (S == 3) RB_CMB(3);
    else RB_CMB(4);
#undef RB_CMB
}

// Back substitution H[0:jf, 0:jf] y = g[0:jf] for replicas active at cycle start, by
// columns with one wavefront per replica: once y_i is known every row above it drops
// its term, read from column i of H (contiguous); the right-hand side lives in LDS.
__global__ __launch_bounds__(64) void k_trisolve(int nrep, int m, const double *H, const double *gv, const int *cyc,
                                                 const int *jf, double *y) {
    const int r = blockIdx.x;
    if (r >= nrep || !cyc[r]) return;
    extern __shared__ double s_rhs[];   // m + 1 entries
    const int n = jf[r], lane = threadIdx.x;
    const double *Hr = H + (long long)r * (m + 1) * m;
    const double *g = gv + (long long)r * (m + 1);
    double *yr = y + (long long)r * (m + 1);
    for (int k = lane; k < n; k += 64) s_rhs[k] = g[k];
    __syncthreads();
    for (int i = n - 1; i >= 0; --i) {
        const double *col = Hr + (long long)i * (m + 1);
        const double d = col[i];
        const double yi = d != 0.0 ? s_rhs[i] / d : 0.0;
        for (int k = lane; k < i; k += 64) s_rhs[k] -= col[k] * yi;   // rows above i only
        if (lane == 0) yr[i] = yi;
        __syncthreads();   // row i - 1 is final before the next step reads it
    }
    for (int i = n + lane; i < m; i += 64) yr[i] = 0.0;
}

// x += sum_{i < jf} y_i Z_i
// (the column loop is unrolled so that eight loads, one basis vector apart, are in
// flight together; the sum keeps its order); Z is FP64, or FP32 with an FP32 preconditioner
template <typename TZ>
__global__ __launch_bounds__(RB_BLOCK) void k_update_x(const RepDev *reps, const BlockEnt *tab,
                                                       const TZ *__restrict__ Z, long long L, int m,
                                                       const double *__restrict__ y, const int *jf, const int *cyc,
                                                       double *__restrict__ x) {
    BlockEnt be = tab[blockIdx.x];
    if (!cyc[be.rep]) return;
    const RepDev &R = reps[be.rep];
    int n = jf[be.rep];
    const double *yr = y + (long long)be.rep * (m + 1);
    long long b = R.off + be.start;
    long long e = R.off + min(be.start + (long long)be.npt * RB_BLOCK, R.len);
    for (long long g = b + threadIdx.x; g < e; g += RB_BLOCK) {
        double acc = 0.0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) acc += yr[i] * (double)Z[(long long)i * L + g];
        x[g] += acc;
    }
}

void launch_trisolve_update(Ctx &c) {
    hipLaunchKernelGGL(k_trisolve, dim3(c.nrep), dim3(64), (size_t)(c.m + 1) * sizeof(double), c.stream, c.nrep,
                       c.m, c.H, c.gv, c.cyc_active, c.jf, c.yv);
    if (c.Zf)
        hipLaunchKernelGGL(k_update_x<float>, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps, c.d_tab_vec,
                           c.Zf, c.L, c.m, c.yv, c.jf, c.cyc_active, c.xsol);
    else
        hipLaunchKernelGGL(k_update_x<double>, dim3(c.n_tab_vec), dim3(RB_BLOCK), 0, c.stream, c.d_reps,
                           c.d_tab_vec, c.Z, c.L, c.m, c.yv, c.jf, c.cyc_active, c.xsol);
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

// Host side of the RB-FIB library: context construction (multigrid hierarchy,
// block tables, dense coarsest-level inverses, body-block data), the batched
// right-preconditioned FGMRES driver, the preconditioner and operator sequences,
// and the C ABI declared in include/rbfib.h.
#include "common.h"

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

static thread_local std::string g_last_error;

void rb_last_hip_error(hipError_t e, const char *what, const char *file, int line) {
    g_last_error = std::string(hipGetErrorString(e)) + " in " + what + " at " + file + ":" + std::to_string(line);
}

struct rbfib_ctx {
    rb::Ctx c;
};

namespace rb {

// ------------------------------------------------------------------ small host linear algebra
// In-place Gauss-Jordan inverse with partial pivoting (n <= ~1000).
static bool invert(std::vector<double> &A, int n) {
    std::vector<int> piv(n);
    std::vector<double> inv(n * (size_t)n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int best = col;
        double bv = std::fabs(A[(size_t)col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            double v = std::fabs(A[(size_t)r * n + col]);
            if (v > bv) { bv = v; best = r; }
        }
        if (bv == 0.0) return false;
        if (best != col) {
            for (int k = 0; k < n; ++k) {
                std::swap(A[(size_t)col * n + k], A[(size_t)best * n + k]);
                std::swap(inv[(size_t)col * n + k], inv[(size_t)best * n + k]);
            }
        }
        double d = 1.0 / A[(size_t)col * n + col];
        for (int k = 0; k < n; ++k) { A[(size_t)col * n + k] *= d; inv[(size_t)col * n + k] *= d; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)col * n + k];
            }
        }
    }
    A.swap(inv);
    return true;
}

// Dense inverse of A = s * Lap on a coarsest grid (component comp, or 3 = pressure),
// padded layout; pinned wall-face slots get zero rows and columns.  The pressure
// operator is singular (constants); its inverse is taken on the mean-zero subspace
// via the matrix bordered by the mean constraint.
static std::vector<double> coarse_inverse(const int n[3], const double ih2[3], const int bc[3], double eta, int comp) {
    int m = n[0] * n[1] * n[2];
    std::vector<int> map(m, -1);
    int nu = 0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int idx[3] = {i, j, k};
                bool pin = comp < 3 && bc[comp] != RBFIB_PERIODIC && idx[comp] == 0;
                if (!pin) map[i + n[0] * (j + n[1] * k)] = nu++;
            }
    bool singular = (comp == 3);
    int nn = nu + (singular ? 1 : 0);
    std::vector<double> A((size_t)nn * nn, 0.0);
    double s = comp < 3 ? -eta : -1.0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int idx[3] = {i, j, k};
                int row = map[i + n[0] * (j + n[1] * k)];
                if (row < 0) continue;
                for (int a = 0; a < 3; ++a) {
                    A[(size_t)row * nn + row] += -2.0 * s * ih2[a];
                    for (int d = -1; d <= 1; d += 2) {
                        int q[3] = {idx[0], idx[1], idx[2]};
                        q[a] += d;
                        if (bc[a] == RBFIB_PERIODIC) {
                            q[a] = (q[a] + n[a]) % n[a];
                        } else if (a == comp) {
                            if (q[a] <= 0 || q[a] >= n[a]) continue;
                        } else if (q[a] < 0 || q[a] >= n[a]) {
                            // even ghost (pressure; tangential velocity at a free-slip
                            // wall) or odd ghost (tangential velocity at a no-slip wall)
                            A[(size_t)row * nn + row] += ((comp == 3 || bc[a] == RBFIB_SLIP) ? 1.0 : -1.0) * s * ih2[a];
                            continue;
                        }
                        int col = map[q[0] + n[0] * (q[1] + n[1] * q[2])];
                        if (col >= 0) A[(size_t)row * nn + col] += s * ih2[a];
                    }
                }
            }
    if (singular) {
        for (int r = 0; r < nu; ++r) { A[(size_t)r * nn + nu] = 1.0; A[(size_t)nu * nn + r] = 1.0; }
    }
    if (!invert(A, nn)) throw (int)RBFIB_EINVAL;
    std::vector<double> out((size_t)m * m, 0.0);
    for (int r = 0; r < m; ++r) {
        if (map[r] < 0) continue;
        for (int cc = 0; cc < m; ++cc) {
            if (map[cc] < 0) continue;
            out[(size_t)r * m + cc] = A[(size_t)map[r] * nn + map[cc]];
        }
    }
    return out;
}

// Rotne-Prager-Yamakawa blob mobility (free space), only used to build the body block
// of the preconditioner.
static std::vector<double> rpy_matrix(const double *x, int n, double a, double eta) {
    std::vector<double> M((size_t)9 * n * n, 0.0);
    double c0 = 1.0 / (6.0 * M_PI * eta * a);
    int N3 = 3 * n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
            double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) {
                    double I = (p == q) ? 1.0 : 0.0;
                    double v;
                    if (i == j) v = c0 * I;
                    else {
                        double e = d[p] * d[q] / (r * r);
                        if (r >= 2 * a)
                            v = (1.0 / (8.0 * M_PI * eta * r)) * ((1 + 2 * a * a / (3 * r * r)) * I + (1 - 2 * a * a / (r * r)) * e);
                        else
                            v = c0 * ((1 - 9 * r / (32 * a)) * I + (3 * r / (32 * a)) * e);
                    }
                    M[(size_t)(3 * i + p) * N3 + 3 * j + q] = v;
                }
        }
    return M;
}

// ------------------------------------------------------------------ allocation helpers
template <typename T>
static T *dalloc(size_t n) {
    if (n == 0) n = 1;
    void *p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
        g_last_error = "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed";
        throw (int)RBFIB_ENOMEM;
    }
    return reinterpret_cast<T *>(p);
}

template <typename T>
static T *upload(Ctx &c, const std::vector<T> &h) {
    T *d = dalloc<T>(h.size());
    if (!h.empty()) HIP_OK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c.stream));
    return d;
}

template <typename T>
void zero_device(Ctx &c, T *p, long long n) {
    if (n > 0) HIP_OK(hipMemsetAsync(p, 0, (size_t)n * sizeof(T), c.stream));
}

static void free_all(Ctx &c);

// Captured FGMRES iterations bake in the tolerance and the multigrid settings;
// they are rebuilt on the next solve after any of these change.
static void drop_graphs(Ctx &c) {
    for (int f = 0; f < 2; ++f)
        for (auto &g : c.graphs[f]) if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// ------------------------------------------------------------------ operator and preconditioner
// Events around one launch of a timed kernel class; `bytes` (given with the
// closing record) is the launch's algorithmic HBM traffic.
static void record(Ctx &c, int cls, bool start, double bytes = 0.0) {
    if (!c.timing.on) return;
    auto &v = c.timing.ev[cls];
    size_t k = c.timing.used[cls];
    if (start) {
        if (k + 2 > v.size()) return;
        HIP_OK(hipEventRecord(v[k], c.stream));
    } else {
        if (k + 2 > v.size()) return;
        HIP_OK(hipEventRecord(v[k + 1], c.stream));
        c.timing.ev_bytes[cls][k / 2] = bytes;
        c.timing.used[cls] = k + 2;
    }
}

// Algorithmic bytes of one spreading pass into a state vector (timing runs only; reads
// the active-tile count back): the read-modify-write of the three FP64 velocity
// components on every cell of every target tile, plus each marker's position and
// lambda (lam_size bytes per value).
static double spread_bytes(Ctx &c, MarkerSet &ms, size_t lam_size) {
    int na = 0;
    HIP_OK(hipMemcpyAsync(&na, ms.n_active, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return (double)na * 64.0 * 3.0 * 16.0 + (double)c.nm * (24.0 + 3.0 * lam_size);
}

// y = A x; x is FP64, or FP32 for the preconditioned vectors of an FP32 preconditioner
template <typename TX>
static void apply_op(Ctx &c, MarkerSet &ms, const TX *x, double *y, bool fluid_only) {
    record(c, 0, true);
    launch_apply_fluid(c, x, y);
    record(c, 0, false, c.cells_all * (4.0 * sizeof(TX) + 32.0));   // read 4 fields of x, write 4 FP64
    if (fluid_only || c.nm == 0) {
        launch_zero_bodies(c, y);
        return;
    }
    const double sb = c.timing.on ? spread_bytes(c, ms, sizeof(TX)) : 0.0;   // before the events
    record(c, 6, true);
    launch_spread(c, ms, x, y, -1.0);
    record(c, 6, false, sb);
    launch_body_apply(c, ms, nullptr, x, y);
}

// One V-cycle on components c0 .. c0+nc-1 of the multigrid pools; returns the
// pool that holds the level-0 result.  Each level runs either the fused down/up
// kernels (two sweeps only, and enough workgroups to fill the device) or the
// separate smoother / restriction / prolongation kernels; both give the same
// values.  After the down pass X holds each level's smoothed iterate and B its
// right-hand side; the corrected result of level l ends in res[l] (T after a
// fused up pass, X after a separate one), where the coarse solve of the
// replicas whose coarsest level is l also writes.
template <typename T>
static T *vcycle(Ctx &c, int c0, int nc) {
    T *X = (T *)c.mg_x, *B = (T *)c.mg_b, *Tt = (T *)c.mg_t;
    const double sz = (double)sizeof(T) * nc;
    // pressure cycles (c0 == 3) may use their own sweep count
    const int nu = std::max(1, (c0 == 3 && c.opts.mg_sweeps_p > 0) ? c.opts.mg_sweeps_p : c.opts.mg_sweeps);
    // weight of sweep k = 1 .. nu: mg_omega, or with mg_cheby = a > 0 the reciprocals
    // of the roots of the degree-nu Chebyshev polynomial on [a, 2], the interval of
    // the high-frequency eigenvalues of D^-1 A that the sweeps must damp
    SweepW sw;
    for (int k = 1; k <= RB_MAXSWEEP; ++k) {
        double w = c.opts.mg_omega;
        if (c.opts.mg_cheby > 0.0 && k <= nu) {
            const double a = c.opts.mg_cheby, b = 2.0;
            w = 1.0 / (0.5 * (b + a) + 0.5 * (b - a) * std::cos((2.0 * k - 1.0) * M_PI / (2.0 * nu)));
        }
        sw.w[k - 1] = w;
    }
    auto omega = [&](int k) { return sw.w[k - 1]; };
    bool fz[RB_MAXLEV];
    T *res[RB_MAXLEV];
    for (int l = 0; l < c.maxlev; ++l) {
        fz[l] = nu == 2 && l + 1 < c.maxlev &&
                (c.opts.mg_fused == 2 || (c.opts.mg_fused == 1 && (long long)c.n_tab_mg[l] * nc >= MGF_MIN_BLOCKS));
        // separate kernels: the up sweeps alternate X -> T -> X ..., ending in T for odd counts
        res[l] = (fz[l] || nu % 2 == 1) ? Tt : X;
    }
    for (int l = 0; l < c.maxlev; ++l) {
        launch_coarse<T>(c, l, c0, nc, B, res[l]);
        if (c.n_tab_lev[l] == 0) continue;
        if (fz[l]) {
            if (l == 0) record(c, 2, true);
            launch_mg_down<T>(c, l, c0, nc, B, X, omega(1), omega(2));
            if (l == 0) record(c, 2, false, sz * (2.0 * c.lev_cells[0] + c.lev_cells_c[0]));
            continue;
        }
        for (int k = 1; k <= nu; ++k) {
            T *out = ((nu - k) % 2 == 0) ? X : Tt;
            T *in = (out == X) ? Tt : X;
            if (l == 0) record(c, 1, true);
            if (k == 1 && nu >= 2 && c.opts.mg_first2 &&
                launch_smooth_first2<T>(c, l, c0, nc, ((nu - 2) % 2 == 0) ? X : Tt, B, omega(1), omega(2))) {
                if (l == 0) record(c, 1, false, sz * c.lev_cells[0] * 2.0);
                ++k;   // sweeps 1 and 2 done
                continue;
            }
            launch_smooth<T>(c, l, c0, nc, in, out, B, k == 1, omega(k));
            if (l == 0) record(c, 1, false, sz * c.lev_cells[0] * (k == 1 ? 2.0 : 3.0));
        }
        launch_restrict<T>(c, l, c0, nc, X, B, B, Tt);   // T(l) is free after the down sweeps
    }
    // levels lb .. nlev-1 of every replica in one launch; its result lands in res[lb]
    unsigned res_t = 0;
    for (int l = 0; l < c.maxlev; ++l) res_t |= (res[l] == Tt ? 1u : 0u) << l;
    launch_mg_bottom<T>(c, c0, nc, nu, sw, B, X, Tt, res_t);
    for (int l = c.maxlev - 2; l >= 0; --l) {
        if (c.n_tab_lev[l] == 0) continue;
        if (fz[l]) {
            if (l == 0) record(c, 3, true);
            launch_mg_up<T>(c, l, c0, nc, B, X, res[l + 1], Tt, omega(1), omega(2));
            if (l == 0) record(c, 3, false, sz * (3.0 * c.lev_cells[0] + c.lev_cells_c[0]));
            continue;
        }
        launch_prolong<T>(c, l, c0, nc, res[l + 1], X);
        T *in = X, *out = Tt;
        for (int k = 1; k <= nu; ++k) {
            if (l == 0) record(c, 1, true);
            launch_smooth<T>(c, l, c0, nc, in, out, B, false, omega(k));
            if (l == 0) record(c, 1, false, sz * c.lev_cells[0] * 3.0);
            std::swap(in, out);
        }
        // the last sweep wrote `in`, which is res[l] by construction
    }
    return res[0];
}

// z = P^-1 (f r), f = rs[rep * (m + 1)] per replica (1 without rs): the readers of r
// apply the factor, so that an unnormalised Krylov vector needs no scaling pass.  z is
// FP64, or FP32 (the FGMRES basis Z of an FP32 preconditioner: A is applied to the
// stored values, so the Arnoldi relation holds for them exactly).
template <typename T, typename TZ>
static void precond_t(Ctx &c, MarkerSet &ms, const double *theta, const double *r, TZ *z, bool fluid_only,
                      const double *rs) {
    bool bodies = !fluid_only && c.nb > 0;
    if (bodies) launch_body_precond(c, ms, theta, r, z, rs);
    // Velocity right-hand side r_v + S lambda built straight in level 0 of the pool;
    // the divergence step reads only the pressure part of r, which spreading leaves alone.
    T *B = (T *)c.mg_b;
    launch_to_level0<T>(c, r, B, 0, 3, rs);
    if (bodies) launch_spread_level0<T>(c, ms, z, B, 1.0);
    T *V = vcycle<T>(c, 0, 3);
    launch_proj_div<T>(c, V, r, B, z, rs);
    T *P = vcycle<T>(c, 3, 1);
    launch_proj_correct<T>(c, V, P, z);
    if (!bodies) launch_zero_bodies(c, z);
    HIP_OK(hipGetLastError());     // a launch the runtime refused surfaces here, not as stale results
}

template <typename TZ>
static void precond(Ctx &c, MarkerSet &ms, const double *theta, const double *r, TZ *z, bool fluid_only,
                    const double *rs = nullptr) {
    if (c.mg_fp32) precond_t<float, TZ>(c, ms, theta, r, z, fluid_only, rs);
    else if constexpr (sizeof(TZ) == 8) precond_t<double, TZ>(c, ms, theta, r, z, fluid_only, rs);
    else throw (int)RBFIB_EINVAL;   // FP32 z only with the FP32 preconditioner
}

// ------------------------------------------------------------------ FGMRES
// Total state length of the active replicas (timing runs: algorithmic bytes of the
// masked Krylov kernels).  One workgroup; fixed summation order.
__global__ void k_active_len(int nrep, const RepDev *reps, const int *active, long long *out) {
    __shared__ long long part[256];
    long long s = 0;
    for (int r = threadIdx.x; r < nrep; r += blockDim.x) s += active[r] ? reps[r].len : 0;
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int k = 0; k < (int)blockDim.x; ++k) t += part[k];
        *out = t;
    }
}

static double active_len(Ctx &c) {
    hipLaunchKernelGGL(k_active_len, dim3(1), dim3(256), 0, c.stream, c.nrep, c.d_reps, c.active, c.d_active_len);
    long long h = 0;
    HIP_OK(hipMemcpyAsync(&h, c.d_active_len, sizeof(long long), hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return (double)h;
}

__global__ void k_init_solver(int nrep, int *active, int *status, int *iters, const double *beta0) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    status[r] = RBFIB_OK;
    iters[r] = 0;
    active[r] = beta0[r] > 0.0 ? 1 : 0;
    if (!isfinite(beta0[r])) { status[r] = RBFIB_ENUMERIC; active[r] = 0; }
}

__global__ void k_count(int nrep, const int *active, int *out) {
    int s = 0;
    for (int r = 0; r < nrep; ++r) s += active[r];
    *out = s;
}

__global__ void k_recheck(int nrep, const double *resid, const double *beta0, double tol, int *active,
                          const int *status) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep || status[r] != RBFIB_OK || active[r]) return;
    if (beta0[r] > 0.0 && resid[r] > tol * beta0[r]) active[r] = 1;
}

static int count_active(Ctx &c) {
    hipLaunchKernelGGL(k_count, dim3(1), dim3(1), 0, c.stream, c.nrep, c.active, c.d_count);
    HIP_OK(hipMemcpyAsync(c.h_count, c.d_count, sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    return *c.h_count;
}

// Solves A x = b (b a state vector); the solution is left in c.xsol.
static void fgmres(Ctx &c, MarkerSet &ms, const double *theta, const double *b, bool fluid_only,
                   std::vector<rbfib_info> &info) {
    const double tol = c.opts.tol;
    const int m = c.m;
    double *nrm = c.hcol + 2LL * c.nrep * (m + 1);
    double *h1 = c.hcol, *h2 = c.hcol + (long long)c.nrep * (m + 1);
    launch_zero(c, c.xsol, nullptr);
    launch_norm(c, b, c.beta0, nullptr);
    hipLaunchKernelGGL(k_init_solver, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.active, c.status,
                       c.iters, c.beta0);
    launch_scale(c, b, c.beta0, c.V, c.active, true);
    HIP_OK(hipMemcpyAsync(nrm, c.beta0, sizeof(double) * c.nrep, hipMemcpyDeviceToDevice, c.stream));
    launch_start_cycle(c);
    int total = 0;
    int check = std::max(1, c.opts.check_every);
    bool done = count_active(c) == 0;
    zero_device(c, h2, (long long)c.nrep * (m + 1));
    const bool reorth = tol < 1e-9;
    // Arnoldi steps per block (krylov_s; single steps with the second Gram-Schmidt pass
    // of tight tolerances); a last block shorter than that runs single steps
    const int sb = reorth ? 1 : std::max(1, std::min(c.opts.krylov_s, RB_MAXS));
    const int check_blocks = std::max(1, check / sb);
    while (true) {
        while (!done) {
            for (int j = 0; j < m; j += (j + sb <= m ? sb : 1)) {
                const int sj = j + sb <= m ? sb : 1;   // steps in this block
                // one Arnoldi step: z_j = P^-1 v_j, w = A z_j, classical Gram-Schmidt
                // (one pass), ||w||, Givens update.  The basis is kept unnormalised:
                // slot i holds u_i with v_i = inv_nu[i] u_i, so w is formed in slot j+1,
                // orthogonalised there, and its norm only enters inv_nu (set by the
                // Givens kernel); the projections, the update coefficients and the
                // preconditioner's reads of v_j apply the factors.  Loss of
                // orthogonality is caught by the true-residual check below.
                auto body_s = [&]() {
                    // s-step block: u_1 = A P^-1 v_j, u_{k+1} = A P^-1 u_k in slots j+1 ..
                    // j+sj, one projection pass and one update pass for all of them, the
                    // Cholesky QR of their Gram matrix in the Givens kernel, then the
                    // combine pass that makes slot j+k the k-th new direction
                    double *W = c.V + (long long)(j + 1) * c.L;
                    c.mask = c.timing.on ? nullptr : c.active;
                    for (int k = 0; k < sj; ++k) {
                        const double *src = c.V + (long long)(j + k) * c.L;
                        double *dst = c.V + (long long)(j + k + 1) * c.L;
                        const double *rs = k == 0 ? c.inv_nu + j : nullptr;
                        if (c.Zf) {
                            float *zk = c.Zf + (long long)(j + k) * c.L;
                            precond(c, ms, theta, src, zk, fluid_only, rs);
                            apply_op(c, ms, zk, dst, fluid_only);
                        } else {
                            double *zk = c.Z + (long long)(j + k) * c.L;
                            precond(c, ms, theta, src, zk, fluid_only, rs);
                            apply_op(c, ms, zk, dst, fluid_only);
                        }
                    }
                    c.mask = nullptr;
                    const double vb = c.timing.on ? 8.0 * active_len(c) : 0.0;
                    record(c, 4, true);
                    launch_block_dots(c, sj, c.V, j + 1, W, c.active, c.inv_nu);
                    record(c, 4, false, vb * (j + 1 + sj));      // read j+1 basis vectors and sj new ones
                    record(c, 5, true);
                    launch_block_update(c, sj, c.V, j + 1, W, c.active, c.inv_nu);
                    record(c, 5, false, vb * (j + 1 + 2 * sj));  // read j+1 vectors and sj, write sj
                    launch_givens_s(c, j, sj, tol);
                    launch_combine_s(c, sj, W, c.active);
                };
                auto body = [&]() {
                    if (sj > 1) { body_s(); return; }
                    double *Vj = c.V + (long long)j * c.L;
                    double *W = c.V + (long long)(j + 1) * c.L;
                    // converged replicas skip the grid and body kernels (not in timing
                    // runs, whose byte counts assume every replica is processed)
                    c.mask = c.timing.on ? nullptr : c.active;
                    if (c.Zf) {
                        float *Zj = c.Zf + (long long)j * c.L;
                        precond(c, ms, theta, Vj, Zj, fluid_only, c.inv_nu + j);
                        apply_op(c, ms, Zj, W, fluid_only);
                    } else {
                        double *Zj = c.Z + (long long)j * c.L;
                        precond(c, ms, theta, Vj, Zj, fluid_only, c.inv_nu + j);
                        apply_op(c, ms, Zj, W, fluid_only);
                    }
                    c.mask = nullptr;
                    // algorithmic bytes of the masked Krylov kernels: FP64 vectors of the active replicas
                    const double vb = c.timing.on ? 8.0 * active_len(c) : 0.0;
                    record(c, 4, true);
                    launch_dots(c, c.V, j + 1, W, h1, c.active, c.inv_nu);
                    record(c, 4, false, vb * (j + 2));    // read j+1 basis vectors and w
                    if (reorth) {
                        // tight tolerances: second Gram-Schmidt pass keeps the basis
                        // orthogonal to working precision
                        launch_axpy_multi(c, c.V, j + 1, h1, W, -1.0, c.active, c.inv_nu);
                        launch_dots(c, c.V, j + 1, W, h2, c.active, c.inv_nu);
                        launch_axpy_multi_norm(c, c.V, j + 1, h2, W, nrm, c.active, c.inv_nu);
                    } else {
                        record(c, 5, true);
                        launch_axpy_multi_norm(c, c.V, j + 1, h1, W, nrm, c.active, c.inv_nu);
                        record(c, 5, false, vb * (j + 3));    // read j+1 vectors and w, write w
                    }
                    launch_givens(c, j, tol);
                };
                bool graphable = c.opts.use_graphs && !c.timing.on && theta == c.theta_int && &ms == &c.ms[0];
                if (graphable) {
                    if (c.graph_tol != tol) {
                        drop_graphs(c);
                        c.graph_tol = tol;
                    }
                    hipGraphExec_t &ge = c.graphs[fluid_only ? 1 : 0][j];
                    if (!ge) {
                        hipGraph_t gr;
                        HIP_OK(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
                        body();
                        HIP_OK(hipStreamEndCapture(c.stream, &gr));
                        HIP_OK(hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0));
                        (void)hipGraphDestroy(gr);
                    }
                    HIP_OK(hipGraphLaunch(ge, c.stream));
                } else {
                    body();
                }
                total += sj;
                if ((j / sb + 1) % check_blocks == 0 || j + sj == m || total >= c.opts.max_iter) {
                    if (count_active(c) == 0) { done = true; break; }
                    if (total >= c.opts.max_iter) break;
                }
            }
            launch_trisolve_update(c);
            if (done || total >= c.opts.max_iter) break;
            // restart for replicas still active: r = b - A x
            apply_op(c, ms, c.xsol, c.W, fluid_only);
            launch_axpby(c, 1.0, b, -1.0, c.W, c.W, c.active);
            launch_norm(c, c.W, nrm, c.active);
            launch_scale(c, c.W, nrm, c.V, c.active, true);
            launch_start_cycle(c);
        }
        // true residual of every replica; replicas whose Arnoldi estimate was too
        // optimistic are reactivated and restarted from their current iterate
        apply_op(c, ms, c.xsol, c.W, fluid_only);
        launch_axpby(c, 1.0, b, -1.0, c.W, c.W, nullptr);
        launch_norm(c, c.W, c.d_resid, nullptr);
        if (total >= c.opts.max_iter) break;
        hipLaunchKernelGGL(k_recheck, dim3((c.nrep + 63) / 64), dim3(64), 0, c.stream, c.nrep, c.d_resid, c.beta0,
                           tol, c.active, c.status);
        if (count_active(c) == 0) break;
        HIP_OK(hipMemcpyAsync(nrm, c.d_resid, sizeof(double) * c.nrep, hipMemcpyDeviceToDevice, c.stream));
        launch_scale(c, c.W, nrm, c.V, c.active, true);
        launch_start_cycle(c);
        done = false;
    }
    std::vector<double> res(c.nrep), b0(c.nrep);
    std::vector<int> st(c.nrep), it(c.nrep), act(c.nrep);
    HIP_OK(hipMemcpyAsync(res.data(), c.d_resid, sizeof(double) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(b0.data(), c.beta0, sizeof(double) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(st.data(), c.status, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(it.data(), c.iters, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipMemcpyAsync(act.data(), c.active, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    info.resize(c.nrep);
    for (int r = 0; r < c.nrep; ++r) {
        info[r].iters = it[r];
        info[r].rel_residual = b0[r] > 0.0 ? res[r] / b0[r] : 0.0;
        int s = st[r];
        if (s == RBFIB_OK && act[r]) s = RBFIB_ENOCONV;
        if (s == RBFIB_OK && !(info[r].rel_residual == info[r].rel_residual)) s = RBFIB_ENUMERIC;
        info[r].status = s;
    }
    if (c.timing.on) {
        for (int cls = 0; cls < RB_NTIMING; ++cls) {
            for (size_t k = 0; k + 1 < c.timing.used[cls]; k += 2) {
                float ms_ = 0.f;
                HIP_OK(hipEventElapsedTime(&ms_, c.timing.ev[cls][k], c.timing.ev[cls][k + 1]));
                c.timing.total_ms[cls] += ms_;
                c.timing.bytes[cls] += c.timing.ev_bytes[cls][k / 2];
                c.timing.launches[cls] += 1;
            }
            c.timing.used[cls] = 0;
        }
    }
}

static int first_bad(const std::vector<rbfib_info> &info) {
    for (auto &i : info) if (i.status != RBFIB_OK) return i.status;
    return RBFIB_OK;
}

// Per-replica flags (bit 0: a marker outside the open domain along a wall axis,
// bit 1: two body centres closer than opts.min_body_dist, bit 2: a solve of the step
// failed, bit 3: an orientation that is not a unit quaternion to 1e-12).
static void clear_flags(Ctx &c) { HIP_OK(hipMemsetAsync(c.d_flags, 0, sizeof(int) * c.nrep, c.stream)); }

static bool read_flags(Ctx &c) {
    HIP_OK(hipMemcpyAsync(c.h_flags, c.d_flags, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    bool any = false;
    for (int r = 0; r < c.nrep; ++r) any |= c.h_flags[r] != 0;
    return any;
}

// Markers at (q, theta) into ms.  Caller-supplied configurations are validated:
// RBFIB_EINVAL when an orientation is not a unit quaternion to 1e-12, and with
// check_domain RBFIB_EREJECT when a marker lies outside the open domain along a wall
// axis.  Both read the flags back, so they synchronise the stream.
static int build_markers(Ctx &c, MarkerSet &ms, const double *q, const double *theta, bool check_domain) {
    clear_flags(c);
    launch_markers(c, ms, q, theta);
    if (c.nb == 0 || !read_flags(c)) return RBFIB_OK;
    bool inval = false, outside = false;
    for (int r = 0; r < c.nrep; ++r) {
        inval |= (c.h_flags[r] & 8) != 0;
        outside |= (c.h_flags[r] & 1) != 0;
    }
    if (inval) {
        g_last_error = "an orientation is not a unit quaternion to 1e-12";
        return RBFIB_EINVAL;
    }
    return (check_domain && outside) ? RBFIB_EREJECT : RBFIB_OK;
}

__global__ void k_add_lambda_bc(const RepDev *reps, const int *marker_body, const int *body_rep, int nm,
                                const double *jbc, double *b) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nm) return;
    int m = t / 3, cc = t % 3;
    const RepDev &R = reps[body_rep[marker_body[m]]];
    b[R.off + 4 * R.N + 3LL * (m - R.m0) + cc] += jbc[t];
}

static void add_boundary_terms(Ctx &c, MarkerSet &ms, double *b) {
    bool any = false;
    for (auto &R : c.reps) any |= (R.movwall != 0);
    if (!any) return;
    launch_wall_rhs(c, b);
    if (c.nm > 0) {
        zero_device(c, c.jbc, 3LL * c.nm);
        launch_interp_bc(c, ms, c.jbc, 1.0);
        hipLaunchKernelGGL(k_add_lambda_bc, dim3((3 * c.nm + 255) / 256), dim3(256), 0, c.stream, c.d_reps,
                           c.d_marker_body, c.d_body_rep, c.nm, c.jbc, b);
    }
}

// Copy of the orientations read by the preconditioner (fixed address, so the
// captured FGMRES iterations can be replayed for any caller buffer).
static const double *stage_theta(Ctx &c, const double *theta) {
    if (c.nb > 0)
        HIP_OK(hipMemcpyAsync(c.theta_int, theta, sizeof(double) * 4 * c.nb, hipMemcpyDeviceToDevice, c.stream));
    return c.theta_int;
}

// One SEM step for every replica (Algorithm 1); see include/rbfib.h.
static int sem_step(Ctx &c, double *q, double *theta, const double *FT, const double *slip, double kT, double dt,
                    uint64_t seed, uint64_t step, double *U, std::vector<rbfib_info> &out) {
    const double delta = c.opts.rfd_delta;
    out.assign(c.nrep, rbfib_info{0, 0.0, RBFIB_OK});
    // configuration Q^n must be valid
    const int st0 = build_markers(c, c.ms[0], q, theta, true);
    if (st0 != RBFIB_OK) {
        for (int r = 0; r < c.nrep; ++r)
            if (c.h_flags[r]) out[r].status = (c.h_flags[r] & 8) ? RBFIB_EINVAL : RBFIB_EREJECT;
        return st0;
    }
    std::vector<rbfib_info> inf;
    const double *th_solve = stage_theta(c, theta);
    // 1. random forces/torques and displaced configurations
    launch_body_rfd(c, kT, delta, seed, step, q, theta);
    const bool drift = c.opts.no_drift == 0;
    // 2. RFD solve: force W^FT, homogeneous data (naive scheme: x^R = 0)
    if (drift) {
        launch_zero(c, c.rhs, nullptr);
        launch_set_rhs_U(c, c.WFT, c.rhs);
        fgmres(c, c.ms[0], th_solve, c.rhs, false, inf);
        for (int r = 0; r < c.nrep; ++r) { out[r].iters += inf[r].iters; if (inf[r].status) out[r].status = inf[r].status; }
        HIP_OK(hipMemcpyAsync(c.xR, c.xsol, sizeof(double) * c.L, hipMemcpyDeviceToDevice, c.stream));
    } else {
        zero_device(c, c.xR, c.L);
    }
    // 3. markers at Q+ and Q- (also for the rejection test of step 7)
    clear_flags(c);
    launch_markers(c, c.ms[1], c.q_buf[0], c.th_buf[0]);
    launch_markers(c, c.ms[2], c.q_buf[1], c.th_buf[1]);
    // 4. unconstrained Stokes solve with (1/delta)[S(Q+) - S(Q-)] lambda^R (naive scheme: v# = 0)
    if (drift) {
        launch_zero(c, c.rhs, nullptr);
        launch_spread(c, c.ms[1], c.xR, c.rhs, 1.0 / delta);
        launch_spread(c, c.ms[2], c.xR, c.rhs, -1.0 / delta);
        fgmres(c, c.ms[0], th_solve, c.rhs, true, inf);
        for (int r = 0; r < c.nrep; ++r) { out[r].iters += inf[r].iters; if (inf[r].status) out[r].status = inf[r].status; }
        HIP_OK(hipMemcpyAsync(c.xS, c.xsol, sizeof(double) * c.L, hipMemcpyDeviceToDevice, c.stream));
    } else {
        zero_device(c, c.xS, c.L);
    }
    // 5. random finite differences of K, J (markers) and K^T (bodies)
    launch_rfd_terms(c, delta);
    launch_rfd_forces(c, delta, FT);
    // 6. noisy constrained solve with the drift terms
    launch_zero(c, c.rhs, nullptr);
    if (kT > 0.0) launch_noise(c, kT, dt, seed, step, c.rhs, false);
    launch_sem_rhs_lambda(c, slip, c.rhs);
    launch_set_rhs_U(c, c.Fp, c.rhs);
    add_boundary_terms(c, c.ms[0], c.rhs);
    fgmres(c, c.ms[0], th_solve, c.rhs, false, inf);
    for (int r = 0; r < c.nrep; ++r) {
        out[r].iters += inf[r].iters;
        out[r].rel_residual = inf[r].rel_residual;
        if (inf[r].status) out[r].status = inf[r].status;
    }
    if (U) launch_copy_U(c, c.xsol, U, 1.0);
    // 7. update and rejection (Q+-, Q^{n+1} outside, or bodies too close)
    launch_update_positions(c, q, theta, c.xsol, dt);
    launch_markers(c, c.ms[3], c.q_buf[2], c.th_buf[2]);
    launch_body_distance(c, c.opts.min_body_dist);
    // replicas whose solves failed keep their state as well
    std::vector<int> bad(c.nrep, 0);
    for (int r = 0; r < c.nrep; ++r) bad[r] = out[r].status != RBFIB_OK ? 4 : 0;
    bool anybad = false;
    for (int r = 0; r < c.nrep; ++r) anybad |= bad[r] != 0;
    if (anybad) {
        HIP_OK(hipMemcpyAsync(c.h_flags, c.d_flags, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        for (int r = 0; r < c.nrep; ++r) c.h_flags[r] |= bad[r];
        HIP_OK(hipMemcpyAsync(c.d_flags, c.h_flags, sizeof(int) * c.nrep, hipMemcpyHostToDevice, c.stream));
    }
    launch_commit_positions(c, q, theta);
    read_flags(c);
    int ret = RBFIB_OK;
    for (int r = 0; r < c.nrep; ++r) {
        if (c.h_flags[r] & 3) out[r].status = RBFIB_EREJECT;
        if (out[r].status != RBFIB_OK && ret == RBFIB_OK) ret = out[r].status;
    }
    return ret;
}

// ------------------------------------------------------------------ context construction
static void validate(int nrep, const rbfib_grid *grids, const rbfib_bodies *bodies, const rbfib_opts &o) {
    if (nrep < 1 || !grids || !bodies) throw (int)RBFIB_EINVAL;
    if (!(o.tol > 0.0) || o.restart < 1 || o.restart > 200 || o.max_iter < 1 || o.mg_sweeps < 1 ||
        !(o.mg_omega > 0.0) || !(o.blob_radius > 0.0) || !(o.rfd_delta > 0.0) || o.mg_bottom < 0 || o.mg_bottom > MGB_LDS / 1024 ||
        !(o.mg_cheby >= 0.0 && o.mg_cheby < 2.0) || o.mg_sweeps > RB_MAXSWEEP || o.mg_sweeps_p < 0 ||
        o.mg_sweeps_p > RB_MAXSWEEP || o.krylov_s < 1 || o.krylov_s > RB_MAXS || (o.mg_first2 != 0 && o.mg_first2 != 1) ||
        (o.kernel != 4 && o.kernel != 6) || (o.no_drift != 0 && o.no_drift != 1))
        throw (int)RBFIB_EINVAL;
    for (int r = 0; r < nrep; ++r) {
        const rbfib_grid &g = grids[r];
        int walls = 0, periodic = 0;
        for (int a = 0; a < 3; ++a) {
            if (g.n[a] < 4 || g.n[a] > (1 << 16)) throw (int)RBFIB_EINVAL;
            if ((double)g.n[0] * g.n[1] * g.n[2] >= 2147483647.0) throw (int)RBFIB_EINVAL;
            if (g.bc[a] != RBFIB_PERIODIC && g.bc[a] != RBFIB_WALL && g.bc[a] != RBFIB_SLIP) throw (int)RBFIB_EINVAL;
            walls += g.bc[a] == RBFIB_WALL;
            periodic += g.bc[a] == RBFIB_PERIODIC;
        }
        // a periodic axis needs a no-slip wall somewhere, or uniform flow along it is free
        if ((walls == 0 && periodic > 0) || periodic == 3 || !(g.h > 0.0) || !(g.eta > 0.0)) throw (int)RBFIB_EINVAL;
        const rbfib_bodies &b = bodies[r];
        if (b.nb < 0 || b.nm < 0) throw (int)RBFIB_EINVAL;
        if (b.nb > 0 && (!b.marker_offset || !b.r_ref)) throw (int)RBFIB_EINVAL;
        if (b.nb > 0) {
            if (b.marker_offset[0] != 0 || b.marker_offset[b.nb] != b.nm) throw (int)RBFIB_EINVAL;
            for (int p = 0; p < b.nb; ++p)
                if (b.marker_offset[p + 1] <= b.marker_offset[p]) throw (int)RBFIB_EINVAL;
        } else if (b.nm != 0) throw (int)RBFIB_EINVAL;
    }
}

// ------------------------------------------------------------------ launch-geometry table
// The autotuner (paper_1901_06427_amd/autotune.py) writes one line per workload class:
//     cells_lo cells_hi reps_lo reps_hi krylov_chunk spread_grid spread_p mg_npt
// ('#' starts a comment).  A context takes the first line whose ranges (inclusive)
// hold its total cell count and replica count.  The file is $RBFIB_TUNING when set
// (empty: built-in defaults), else tuning.txt beside the library; without a file or
// a matching line the built-in defaults apply.  Invalid values are ignored.
static std::string library_dir() {
    Dl_info info;
    if (dladdr((void *)&rbfib_default_opts, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        size_t k = p.find_last_of('/');
        return k == std::string::npos ? std::string(".") : p.substr(0, k);
    }
    return ".";
}

static Tuning load_tuning(long long cells, int nrep, std::string *source) {
    Tuning t;
    const char *env = getenv("RBFIB_TUNING");
    std::string path = env ? std::string(env) : library_dir() + "/tuning.txt";
    if (source) *source = "defaults";
    if (path.empty()) return t;
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return t;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        long long clo, chi;
        int rlo, rhi, ch, sg, sp, np, kc = -1;
        const int got = sscanf(line, "%lld %lld %d %d %d %d %d %d %d", &clo, &chi, &rlo, &rhi, &ch, &sg, &sp, &np, &kc);
        if (got != 8 && got != 9) continue;
        if (cells < clo || cells > chi || nrep < rlo || nrep > rhi) continue;
        if (ch == 512 || ch == 1024 || ch == 2048) t.krylov_chunk = ch;
        if (sg >= 64 && sg <= (1 << 20)) t.spread_grid = sg;
        if (sp == 16 || sp == 32 || sp == 64) t.spread_p = sp;
        if (np == 0 || np == 1 || np == 4) t.mg_npt = np;
        if (kc >= 0 && kc <= 64) t.apply_kc = kc;
        if (source) *source = path;
        break;
    }
    fclose(f);
    return t;
}

static void build(Ctx &c, int nrep, const rbfib_grid *grids, const rbfib_bodies *bodies) {
    c.nrep = nrep;
    c.reps.resize(nrep);
    long long off = 0;
    int b0 = 0, m0 = 0, t0 = 0;
    std::vector<int> marker_body, body_rep, body_off(1, 0), tile_rep;
    std::vector<double> rref;
    c.max_body_nm = 1;
    for (int r = 0; r < nrep; ++r) {
        const rbfib_grid &g = grids[r];
        const rbfib_bodies &bd = bodies[r];
        RepDev &R = c.reps[r];
        memset(&R, 0, sizeof(R));
        rep_from_grid(R, g, bd.nb, bd.nm, off, b0, m0, t0);
        off += R.len;
        int nt = R.tdim[0] * R.tdim[1] * R.tdim[2];
        for (int t = 0; t < nt; ++t) tile_rep.push_back(r);
        t0 += nt;
        for (int p = 0; p < bd.nb; ++p) {
            int n = bd.marker_offset[p + 1] - bd.marker_offset[p];
            c.max_body_nm = std::max(c.max_body_nm, n);
            for (int i = 0; i < n; ++i) marker_body.push_back(b0 + p);
            body_rep.push_back(r);
            body_off.push_back(m0 + bd.marker_offset[p + 1]);
        }
        for (int i = 0; i < 3 * bd.nm; ++i) rref.push_back(bd.r_ref[i]);
        b0 += bd.nb;
        m0 += bd.nm;
    }
    c.L = off; c.nb = b0; c.nm = m0; c.ntiles = t0;

    // ---- multigrid hierarchy: coarsen an axis while it is even and >= 8
    c.levs.assign((size_t)nrep * RB_MAXLEV, LevDev());
    long long loff = 0;
    c.maxlev = 0;
    for (int r = 0; r < nrep; ++r) {
        RepDev &R = c.reps[r];
        int n[3] = {R.n[0], R.n[1], R.n[2]};
        double h[3] = {R.h, R.h, R.h};
        int l = 0;
        while (true) {
            LevDev &Lv = c.levs[(size_t)r * RB_MAXLEV + l];
            for (int a = 0; a < 3; ++a) { Lv.n[a] = n[a]; Lv.inv_h2[a] = 1.0 / (h[a] * h[a]); }
            Lv.N = (long long)n[0] * n[1] * n[2];
            Lv.inv_n0 = 1.0 / n[0];
            Lv.inv_n01 = 1.0 / ((double)n[0] * n[1]);
            Lv.off = loff;
            loff += 4 * Lv.N;
            bool any = false;
            int nn[3];
            for (int a = 0; a < 3; ++a) {
                bool can = (n[a] % 2 == 0) && n[a] >= 8;
                nn[a] = can ? n[a] / 2 : n[a];
                any |= can;
            }
            if (!any || l + 1 >= RB_MAXLEV) break;
            for (int a = 0; a < 3; ++a) { if (nn[a] != n[a]) h[a] *= 2.0; n[a] = nn[a]; }
            ++l;
        }
        R.nlev = l + 1;
        c.maxlev = std::max(c.maxlev, R.nlev);
        if (c.levs[(size_t)r * RB_MAXLEV + l].N > 1000) {
            g_last_error = "coarsest multigrid level has more than 1000 cells; use grid sizes with more factors of 2";
            throw (int)RBFIB_EINVAL;
        }
    }
    c.lev_total = loff;

    // ---- bottom level of each replica: the first level whose grids (x and b of it
    // and every coarser level, plus one scratch grid of its size) fit the LDS budget
    // (mg_bottom KB) of one workgroup; without the bottom kernel only the coarsest
    // level is solved apart
    c.bot_lds32 = c.bot_lds64 = 0;
    for (int r = 0; r < nrep; ++r) {
        RepDev &R = c.reps[r];
        const int lc = R.nlev - 1;
        auto cells = [&](int l) {
            long long n = (l < lc) ? c.levs[(size_t)r * RB_MAXLEV + l].N : 0;
            for (int k = l; k <= lc; ++k) n += 2 * c.levs[(size_t)r * RB_MAXLEV + k].N;
            return n;
        };
        R.lb = lc;
        if (c.opts.mg_bottom) {
            const size_t es = c.opts.precond_fp32 ? sizeof(float) : sizeof(double);
            const size_t budget = (size_t)c.opts.mg_bottom * 1024;
            while (R.lb > 0 && (size_t)cells(R.lb - 1) * es <= budget) --R.lb;
            c.bot_lds32 = std::max(c.bot_lds32, (size_t)cells(R.lb) * sizeof(float));
            c.bot_lds64 = std::max(c.bot_lds64, (size_t)cells(R.lb) * sizeof(double));
        }
    }

    // ---- block tables
    // Grid kernels (level-0 cell kernels and every multigrid level) process npt points
    // per thread: 4 for large batches (amortises the per-block descriptor loads), 1
    // otherwise (keeps enough workgroups in flight on small grids).
    long long total_cells = 0;
    for (int r = 0; r < nrep; ++r) total_cells += c.reps[r].N;
    const int mg_npt = c.tune.mg_npt ? c.tune.mg_npt : (total_cells >= (1LL << 22) ? 4 : 1);
    c.mg_npt = mg_npt;
    // Krylov vector blocks: chunks of krylov_chunk elements, which the block table
    // carries as its points per thread (chunk / RB_BLOCK)
    auto chunks = [](std::vector<BlockEnt> &tab, int rep, long long n, long long step) {
        for (long long s = 0; s < n; s += step) tab.push_back(BlockEnt{rep, (int)(step / RB_BLOCK), s});
    };
    auto gchunks = [](std::vector<BlockEnt> &tab, int rep, long long n, int npt) {
        for (long long s = 0; s < n; s += (long long)RB_BLOCK * npt) tab.push_back(BlockEnt{rep, npt, s});
    };
    std::vector<BlockEnt> tcells, tcells2, tvec;
    c.vec_first.resize(nrep);
    c.vec_nblk.resize(nrep);
    for (int r = 0; r < nrep; ++r) {
        gchunks(tcells, r, c.reps[r].N, mg_npt);
        gchunks(tcells2, r, c.reps[r].N, 2);
        c.vec_first[r] = (int)tvec.size();
        chunks(tvec, r, c.reps[r].len, c.tune.krylov_chunk);
        c.vec_nblk[r] = (int)tvec.size() - c.vec_first[r];
    }
    c.n_tab_cells = (int)tcells.size();
    c.n_tab_vec = (int)tvec.size();
    c.d_tab_cells = upload(c, tcells);
    c.n_tab_cells2 = (int)tcells2.size();
    c.d_tab_cells2 = upload(c, tcells2);
    // z-marching apply: RB_AZT^2 tiles of each x-y plane, apply_kc planes each (x
    // tiles fastest, then y, then z chunks); only when the table asks for it (on the
    // ensemble it is slower than the two-cell apply at every chunk length measured)
    c.apply_kc = c.tune.apply_kc > 0 ? c.tune.apply_kc : 0;
    if (c.apply_kc > 0) {
        std::vector<BlockEnt> taz;
        for (int r = 0; r < nrep; ++r) {
            const RepDev &R = c.reps[r];
            for (int z0 = 0; z0 < R.n[2]; z0 += c.apply_kc)
                for (int y0 = 0; y0 < R.n[1]; y0 += RB_AZT)
                    for (int x0 = 0; x0 < R.n[0]; x0 += RB_AZT)
                        taz.push_back(BlockEnt{r, c.apply_kc, x0 + (long long)R.n[0] * (y0 + (long long)R.n[1] * z0)});
        }
        c.n_tab_az = (int)taz.size();
        c.d_tab_az = upload(c, taz);
    }
    c.d_tab_vec = upload(c, tvec);
    c.d_vec_first = upload(c, c.vec_first);
    c.d_vec_nblk = upload(c, c.vec_nblk);
    // level l of replica r runs in the separate (or fused) kernels for l < lb; the
    // restriction into level l for l <= lb; the coarsest-level kernel only for
    // replicas the bottom kernel does not take
    for (int l = 0; l < c.maxlev; ++l) {
        std::vector<BlockEnt> tl, tc, ta;
        for (int r = 0; r < nrep; ++r) {
            const RepDev &R = c.reps[r];
            if (l >= R.nlev || l > R.lb) continue;
            long long N = c.levs[(size_t)r * RB_MAXLEV + l].N;
            gchunks(ta, r, N, mg_npt);
            if (l < R.lb) gchunks(tl, r, N, mg_npt);
            else if (!c.opts.mg_bottom) tc.push_back(BlockEnt{r, 1, 0});
        }
        c.n_tab_lev[l] = (int)tl.size(); c.d_tab_lev[l] = upload(c, tl);
        bool row4 = true;
        for (const BlockEnt &e : tl) row4 = row4 && c.levs[(size_t)e.rep * RB_MAXLEV + l].n[0] % 4 == 0;
        c.lev_row4[l] = row4;
        c.n_tab_crs[l] = (int)tc.size(); c.d_tab_crs[l] = upload(c, tc);
        c.n_tab_all[l] = (int)ta.size(); c.d_tab_all[l] = upload(c, ta);
    }
    // fused level kernels: one block per MGF_OX x MGF_OY x MGF_ZC block of level l
    for (int l = 0; l + 1 < c.maxlev; ++l) {
        std::vector<BlockEnt> tm;
        for (int r = 0; r < nrep; ++r) {
            if (l >= c.reps[r].lb) continue;
            const LevDev &F = c.levs[(size_t)r * RB_MAXLEV + l];
            const LevDev &C = c.levs[(size_t)r * RB_MAXLEV + l + 1];
            const long long nt = (long long)((F.n[0] + MGF_OX - 1) / MGF_OX) * ((F.n[1] + MGF_OY - 1) / MGF_OY) *
                                 ((F.n[2] + MGF_ZC - 1) / MGF_ZC);
            for (long long t = 0; t < nt; ++t) tm.push_back(BlockEnt{r, 1, t});
            c.lev_cells[l] += (double)F.N;
            c.lev_cells_c[l] += (double)C.N;
        }
        c.n_tab_mg[l] = (int)tm.size(); c.d_tab_mg[l] = upload(c, tm);
    }
    c.cells_all = (double)total_cells;
    if (c.opts.mg_bottom) {
        std::vector<BlockEnt> tb;
        for (int r = 0; r < nrep; ++r) tb.push_back(BlockEnt{r, 1, 0});
        c.n_tab_bot = (int)tb.size();
        c.d_tab_bot = upload(c, tb);
    }

    // ---- dense coarsest inverses, deduplicated by (dims, spacing, bc, eta, component)
    std::map<std::string, long long> keyoff;
    std::vector<double> pool;
    std::vector<long long> coff((size_t)nrep * 4, 0);
    c.max_coarse = 1;
    for (int r = 0; r < nrep; ++r) {
        const RepDev &R = c.reps[r];
        const LevDev &Lv = c.levs[(size_t)r * RB_MAXLEV + R.nlev - 1];
        c.max_coarse = std::max(c.max_coarse, (int)Lv.N);
        for (int comp = 0; comp < 4; ++comp) {
            char key[512];
            snprintf(key, sizeof key, "%d %d %d %.17g %.17g %.17g %d %d %d %.17g %d", Lv.n[0], Lv.n[1], Lv.n[2],
                     Lv.inv_h2[0], Lv.inv_h2[1], Lv.inv_h2[2], R.bc[0], R.bc[1], R.bc[2], R.eta, comp);
            auto it = keyoff.find(key);
            if (it == keyoff.end()) {
                std::vector<double> inv = coarse_inverse(Lv.n, Lv.inv_h2, R.bc, R.eta, comp);
                long long o = (long long)pool.size();
                pool.insert(pool.end(), inv.begin(), inv.end());
                it = keyoff.emplace(key, o).first;
            }
            coff[(size_t)r * 4 + comp] = it->second;
        }
    }
    c.d_coarse64 = upload(c, pool);
    std::vector<float> pool32(pool.begin(), pool.end());
    c.d_coarse32 = upload(c, pool32);
    c.d_coarse_off = upload(c, coff);

    // ---- body shapes for the preconditioner block (deduplicated by marker geometry)
    std::map<std::vector<double>, int> shape_id;
    std::vector<ShapeDev> shapes;
    std::vector<double> sdata;
    std::vector<int> body_shape(c.nb);
    std::vector<double> body_len(c.nb, 0.0);
    for (int p = 0; p < c.nb; ++p) {
        int mb = body_off[p], me = body_off[p + 1], n = me - mb;
        std::vector<double> geo(rref.begin() + 3 * mb, rref.begin() + 3 * me);
        double Lp = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double dx = geo[3 * i] - geo[3 * j], dy = geo[3 * i + 1] - geo[3 * j + 1], dz = geo[3 * i + 2] - geo[3 * j + 2];
                Lp = std::max(Lp, std::sqrt(dx * dx + dy * dy + dz * dz));
            }
        body_len[p] = Lp;
        const RepDev &R = c.reps[body_rep[p]];
        std::vector<double> key = geo;
        key.push_back(R.h);
        key.push_back(R.eta);
        auto it = shape_id.find(key);
        if (it == shape_id.end()) {
            int N3 = 3 * n;
            std::vector<double> M = rpy_matrix(geo.data(), n, c.opts.blob_radius * R.h, R.eta);
            if (!invert(M, N3)) throw (int)RBFIB_EINVAL;
            std::vector<double> K((size_t)N3 * 6, 0.0);
            for (int i = 0; i < n; ++i) {
                const double *d = &geo[3 * i];
                for (int a = 0; a < 3; ++a) K[(size_t)(3 * i + a) * 6 + a] = 1.0;
                // -[d]_x
                K[(size_t)(3 * i + 0) * 6 + 4] = d[2];  K[(size_t)(3 * i + 0) * 6 + 5] = -d[1];
                K[(size_t)(3 * i + 1) * 6 + 3] = -d[2]; K[(size_t)(3 * i + 1) * 6 + 5] = d[0];
                K[(size_t)(3 * i + 2) * 6 + 3] = d[1];  K[(size_t)(3 * i + 2) * 6 + 4] = -d[0];
            }
            std::vector<double> MK((size_t)N3 * 6, 0.0);
            for (int k = 0; k < N3; ++k)
                for (int l = 0; l < 6; ++l) {
                    double s = 0.0;
                    for (int j = 0; j < N3; ++j) s += M[(size_t)k * N3 + j] * K[(size_t)j * 6 + l];
                    MK[(size_t)k * 6 + l] = s;
                }
            std::vector<double> Nm(36, 0.0);
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) {
                    double s = 0.0;
                    for (int j = 0; j < N3; ++j) s += K[(size_t)j * 6 + a] * MK[(size_t)j * 6 + b];
                    Nm[a * 6 + b] = s;
                }
            if (!invert(Nm, 6)) throw (int)RBFIB_EINVAL;
            ShapeDev S;
            S.nm = n;
            S.minv_off = (long long)sdata.size(); sdata.insert(sdata.end(), M.begin(), M.end());
            S.mk_off = (long long)sdata.size(); sdata.insert(sdata.end(), MK.begin(), MK.end());
            S.n_off = (long long)sdata.size(); sdata.insert(sdata.end(), Nm.begin(), Nm.end());
            S.rref_off = (long long)sdata.size(); sdata.insert(sdata.end(), geo.begin(), geo.end());
            shapes.push_back(S);
            it = shape_id.emplace(key, (int)shapes.size() - 1).first;
        }
        body_shape[p] = it->second;
    }

    // ---- device copies
    c.d_reps = upload(c, c.reps);
    c.d_levs = upload(c, c.levs);
    c.d_marker_body = upload(c, marker_body);
    c.d_body_rep = upload(c, body_rep);
    c.d_body_off = upload(c, body_off);
    c.d_tile_rep = upload(c, tile_rep);
    c.d_rref = upload(c, rref);
    c.d_body_shape = upload(c, body_shape);
    c.d_shapes = upload(c, shapes);
    c.d_shape_data = upload(c, sdata);
    c.d_body_len = upload(c, body_len);
    c.h_body_len = body_len;

    // ---- marker sets
    // spreading pairs: at most W/2 tiles per axis per marker (the union of the
    // components' W-point supports spans W + 1 cells), one more on a periodic axis
    // whose last tile is partial, never more than the axis has
    long long pair_cap = 0;
    for (const RepDev &R : c.reps) {
        long long per = 1;
        for (int a = 0; a < 3; ++a) {
            int b = c.kw / 2 + ((R.bc[a] == RBFIB_PERIODIC && R.n[a] % RB_TILE != 0) ? 1 : 0);
            per *= std::min(b, R.tdim[a]);
        }
        pair_cap += per * R.nm;
    }
    pair_cap = std::max(pair_cap, 1LL);
    // tile-start offsets are int: even 64 pairs per marker must fit
    if (64LL * c.nm > 2147483647LL) throw (int)RBFIB_EINVAL;
    for (int k = 0; k < 4; ++k) {
        MarkerSet &ms = c.ms[k];
        ms.r = dalloc<double>(3 * (size_t)c.nm);
        ms.d = dalloc<double>(3 * (size_t)c.nm);
        ms.tile = dalloc<int>(c.nm);
        ms.perm = dalloc<int>(c.nm);
        ms.tile_count = dalloc<int>(c.ntiles);
        ms.tile_start = dalloc<int>(c.ntiles);
        ms.tile_fill = dalloc<int>(c.ntiles);
        ms.active = dalloc<int>(c.ntiles);
        ms.n_active = dalloc<int>(1);
        ms.wc = dalloc<double>(9 * (size_t)c.kw * std::max(c.nm, 1));
        ms.ic = dalloc<int>(9 * (size_t)c.kw * std::max(c.nm, 1));
        ms.pair_cap = pair_cap;
        ms.pair_count = dalloc<int>(c.ntiles);
        ms.pair_start = dalloc<int>(c.ntiles);
        ms.pair_fill = dalloc<int>(c.ntiles);
        ms.pair_m = dalloc<int>(pair_cap);
        ms.pair_tile = dalloc<int>(pair_cap);
        zero_device(c, ms.n_active, 1);
    }
    c.theta_int = dalloc<double>(4 * (size_t)std::max(c.nb, 1));
    c.graphs[0].assign(c.opts.restart, nullptr);
    c.graphs[1].assign(c.opts.restart, nullptr);
    c.d_flags = dalloc<int>(std::max(nrep, 4));
    c.d_scan = dalloc<int>((c.ntiles + 1023) / 1024 + 1);
    HIP_OK(hipHostMalloc((void **)&c.h_flags, sizeof(int) * std::max(nrep, 4), hipHostMallocDefault));
    HIP_OK(hipHostMalloc((void **)&c.h_count, sizeof(int), hipHostMallocDefault));
    c.d_count = dalloc<int>(1);
    c.d_active_len = dalloc<long long>(1);

    // ---- multigrid pools
    c.mg_fp32 = c.opts.precond_fp32 != 0;
    size_t es = c.mg_fp32 ? sizeof(float) : sizeof(double);
    c.mg_x = dalloc<unsigned char>(es * (size_t)c.lev_total);
    c.mg_b = dalloc<unsigned char>(es * (size_t)c.lev_total);
    c.mg_t = dalloc<unsigned char>(es * (size_t)c.lev_total);
    HIP_OK(hipMemsetAsync(c.mg_x, 0, es * (size_t)c.lev_total, c.stream));
    HIP_OK(hipMemsetAsync(c.mg_b, 0, es * (size_t)c.lev_total, c.stream));
    HIP_OK(hipMemsetAsync(c.mg_t, 0, es * (size_t)c.lev_total, c.stream));

    // ---- Krylov storage
    c.m = c.opts.restart;
    size_t L = (size_t)c.L;
    c.V = dalloc<double>(L * (c.m + 1));
    // preconditioned vectors: FP32 with the FP32 preconditioner (half the traffic of the
    // apply's input, of the projection outputs and of the solution update)
    if (c.mg_fp32) c.Zf = dalloc<float>(L * c.m);
    else c.Z = dalloc<double>(L * c.m);
    c.W = dalloc<double>(L);
    c.xsol = dalloc<double>(L);
    c.rhs = dalloc<double>(L);
    c.xR = dalloc<double>(L);
    c.xS = dalloc<double>(L);
    c.partial = dalloc<double>((size_t)c.n_tab_vec * RB_MAXS * (c.m + 1));   // s-step blocks: s (m + 1) per block
    c.H = dalloc<double>((size_t)nrep * (c.m + 1) * c.m);
    c.cs = dalloc<double>((size_t)nrep * c.m);
    c.sn = dalloc<double>((size_t)nrep * c.m);
    c.gv = dalloc<double>((size_t)nrep * (c.m + 1));
    c.beta0 = dalloc<double>(nrep);
    c.hcol = dalloc<double>((size_t)3 * nrep * (c.m + 1));
    c.inv_nu = dalloc<double>((size_t)nrep * (c.m + 1));
    c.hblk = dalloc<double>((size_t)RB_MAXS * nrep * (c.m + 1));
    c.gram = dalloc<double>((size_t)nrep * RB_MAXG);
    c.tco = dalloc<double>((size_t)nrep * RB_MAXS * RB_MAXS);
    zero_device(c, c.inv_nu, (long long)nrep * (c.m + 1));
    c.yv = dalloc<double>((size_t)nrep * (c.m + 1));
    c.d_resid = dalloc<double>(nrep);
    c.active = dalloc<int>(nrep);
    c.cyc_active = dalloc<int>(nrep);
    c.jf = dalloc<int>(nrep);
    c.status = dalloc<int>(nrep);
    c.iters = dalloc<int>(nrep);
    zero_device(c, c.H, (long long)nrep * (c.m + 1) * c.m);
    zero_device(c, c.hcol, 3LL * nrep * (c.m + 1));
    // SEM scratch
    for (int k = 0; k < 3; ++k) {
        c.q_buf[k] = dalloc<double>(3 * (size_t)std::max(c.nb, 1));
        c.th_buf[k] = dalloc<double>(4 * (size_t)std::max(c.nb, 1));
    }
    c.Wf = dalloc<double>(3 * (size_t)std::max(c.nb, 1));
    c.Wt = dalloc<double>(3 * (size_t)std::max(c.nb, 1));
    c.WFT = dalloc<double>(6 * (size_t)std::max(c.nb, 1));
    c.Fp = dalloc<double>(6 * (size_t)std::max(c.nb, 1));
    c.UR = dalloc<double>(6 * (size_t)std::max(c.nb, 1));
    c.trap_q0 = dalloc<double>(3 * (size_t)std::max(c.nb, 1));
    c.trap_th0 = dalloc<double>(4 * (size_t)std::max(c.nb, 1));
    c.trap_q = dalloc<double>(3 * (size_t)std::max(c.nb, 1));
    c.trap_th = dalloc<double>(4 * (size_t)std::max(c.nb, 1));
    c.trap_U = dalloc<double>(18 * (size_t)std::max(c.nb, 1));
    c.slip_acc = dalloc<double>(3 * (size_t)std::max(c.nm, 1));
    c.jbc = dalloc<double>(3 * (size_t)std::max(c.nm, 1));
    for (int cls = 0; cls < RB_NTIMING; ++cls) {
        c.timing.ev[cls].resize(8192);
        c.timing.ev_bytes[cls].assign(4096, 0.0);
        for (auto &e : c.timing.ev[cls]) HIP_OK(hipEventCreate(&e));
    }
    HIP_OK(hipStreamSynchronize(c.stream));
}

static void free_all(Ctx &c) {
    auto F = [](void *p) { if (p) (void)hipFree(p); };
    F(c.d_reps); F(c.d_levs); F(c.d_marker_body); F(c.d_body_rep); F(c.d_body_off); F(c.d_tile_rep); F(c.d_rref);
    F(c.d_body_shape); F(c.d_shapes); F(c.d_shape_data); F(c.d_body_len);
    F(c.d_tab_cells); F(c.d_tab_cells2); F(c.d_tab_az); F(c.d_tab_vec); F(c.d_vec_first); F(c.d_vec_nblk); F(c.d_tab_bot);
    for (int l = 0; l < RB_MAXLEV; ++l) {
        F(c.d_tab_lev[l]); F(c.d_tab_crs[l]); F(c.d_tab_all[l]); F(c.d_tab_mg[l]);
    }
    F(c.d_coarse_off); F(c.d_coarse64); F(c.d_coarse32);
    F(c.mg_x); F(c.mg_b); F(c.mg_t);
    for (int k = 0; k < 4; ++k) {
        MarkerSet &ms = c.ms[k];
        F(ms.r); F(ms.d); F(ms.tile); F(ms.perm); F(ms.tile_count); F(ms.tile_start); F(ms.tile_fill);
        F(ms.active); F(ms.n_active); F(ms.wc); F(ms.ic);
        F(ms.pair_count); F(ms.pair_start); F(ms.pair_fill); F(ms.pair_m); F(ms.pair_tile);
    }
    F(c.d_flags); F(c.d_scan); F(c.d_count); F(c.d_active_len);
    if (c.h_flags) (void)hipHostFree(c.h_flags);
    if (c.h_count) (void)hipHostFree(c.h_count);
    F(c.V); F(c.Z); F(c.Zf); F(c.W); F(c.xsol); F(c.rhs); F(c.xR); F(c.xS); F(c.partial);
    F(c.H); F(c.cs); F(c.sn); F(c.gv); F(c.beta0); F(c.hcol); F(c.inv_nu); F(c.hblk); F(c.gram); F(c.tco); F(c.yv); F(c.d_resid);
    F(c.active); F(c.cyc_active); F(c.jf); F(c.status); F(c.iters);
    for (int k = 0; k < 3; ++k) { F(c.q_buf[k]); F(c.th_buf[k]); }
    F(c.Wf); F(c.Wt); F(c.WFT); F(c.Fp); F(c.UR); F(c.slip_acc); F(c.jbc); F(c.theta_int);
    F(c.trap_q0); F(c.trap_th0); F(c.trap_q); F(c.trap_th); F(c.trap_U);
    for (int f = 0; f < 2; ++f)
        for (auto &g : c.graphs[f]) if (g) (void)hipGraphExecDestroy(g);
    if (c.ev_in) (void)hipEventDestroy(c.ev_in);
    if (c.ev_out) (void)hipEventDestroy(c.ev_out);
    if (c.stream && c.stream != c.user_stream) (void)hipStreamDestroy(c.stream);
    for (int cls = 0; cls < RB_NTIMING; ++cls)
        for (auto &e : c.timing.ev[cls]) (void)hipEventDestroy(e);
}

}  // namespace rb

using namespace rb;

// ====================================================================== C ABI
#define GUARD_BEGIN try {
#define GUARD_END                                          \
    }                                                      \
    catch (int code) { return code; }                      \
    catch (...) { g_last_error = "internal error"; return RBFIB_EDEVICE; }

extern "C" {

void rbfib_default_opts(rbfib_opts *o) {
    if (!o) return;
    o->tol = 1e-6;
    o->restart = 100;
    o->max_iter = 600;
    o->precond_fp32 = 0;
    o->mg_sweeps = 2;
    o->mg_sweeps_p = 3;
    o->mg_omega = 0.9;
    o->blob_radius = 1.2;
    o->rfd_delta = 1e-5;
    o->min_body_dist = 0.0;
    o->check_every = 5;
    o->use_graphs = 1;
    o->mg_fused = 0;
    o->mg_bottom = 32;
    o->mg_cheby = 0.27;
    o->krylov_s = 2;
    o->mg_first2 = 1;
    o->kernel = 4;
    o->no_drift = 0;
}

const char *rbfib_strerror(int code) {
    switch (code) {
        case RBFIB_OK: return "ok";
        case RBFIB_EINVAL: return "invalid argument";
        case RBFIB_EREJECT: return "unphysical configuration (step rejected)";
        case RBFIB_ENOCONV: return "solver did not converge";
        case RBFIB_ENUMERIC: return "NaN or Inf in the solver";
        case RBFIB_EDEVICE: return "HIP runtime error";
        case RBFIB_ENOMEM: return "device allocation failed";
        default: return "unknown error";
    }
}

const char *rbfib_last_error(void) { return g_last_error.c_str(); }

int rbfib_create_batch(int nrep, const rbfib_grid *grids, const rbfib_bodies *bodies, const rbfib_opts *opts,
                       void *hip_stream, rbfib_ctx **out) {
    if (!out) return RBFIB_EINVAL;
    *out = nullptr;
    rbfib_ctx *ctx = nullptr;
    try {
        rbfib_opts o;
        rbfib_default_opts(&o);
        if (opts) o = *opts;
        validate(nrep, grids, bodies, o);
        ctx = new rbfib_ctx();
        ctx->c.user_stream = (hipStream_t)hip_stream;
        HIP_OK(hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&ctx->c.ev_in, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&ctx->c.ev_out, hipEventDisableTiming));
        ctx->c.opts = o;
        ctx->c.kw = o.kernel;
        long long cells = 0;
        for (int r = 0; r < nrep; ++r) cells += (long long)grids[r].n[0] * grids[r].n[1] * grids[r].n[2];
        ctx->c.tune = load_tuning(cells, nrep, nullptr);
        build(ctx->c, nrep, grids, bodies);
        *out = ctx;
        return RBFIB_OK;
    } catch (int code) {
        if (ctx) { free_all(ctx->c); delete ctx; }
        return code;
    } catch (...) {
        if (ctx) { free_all(ctx->c); delete ctx; }
        return RBFIB_EDEVICE;
    }
}

int rbfib_create(const rbfib_grid *grid, const rbfib_bodies *bodies, const rbfib_opts *opts, void *hip_stream,
                 rbfib_ctx **out) {
    return rbfib_create_batch(1, grid, bodies, opts, hip_stream, out);
}

void rbfib_destroy(rbfib_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->c.stream);
    free_all(ctx->c);
    delete ctx;
}

int rbfib_set_opts(rbfib_ctx *ctx, const rbfib_opts *o) {
    if (!ctx || !o) return RBFIB_EINVAL;
    Ctx &c = ctx->c;
    if (!(o->tol > 0.0) || o->max_iter < 1 || o->mg_sweeps < 1 || !(o->mg_omega > 0.0) || !(o->rfd_delta > 0.0) ||
        !(o->mg_cheby >= 0.0 && o->mg_cheby < 2.0) || o->mg_sweeps > RB_MAXSWEEP || o->mg_sweeps_p < 0 ||
        o->mg_sweeps_p > RB_MAXSWEEP || o->krylov_s < 1 || o->krylov_s > RB_MAXS ||
        (o->mg_first2 != 0 && o->mg_first2 != 1) || (o->no_drift != 0 && o->no_drift != 1))
        return RBFIB_EINVAL;
    // fields fixed at creation: restart length, precision, blob radius, bottom kernel, delta kernel
    if (o->restart != c.opts.restart || (o->precond_fp32 != 0) != c.mg_fp32 || o->blob_radius != c.opts.blob_radius ||
        o->mg_bottom != c.opts.mg_bottom || o->kernel != c.kw)
        return RBFIB_EINVAL;
    if (o->mg_sweeps != c.opts.mg_sweeps || o->mg_sweeps_p != c.opts.mg_sweeps_p || o->mg_omega != c.opts.mg_omega ||
        o->mg_cheby != c.opts.mg_cheby || o->krylov_s != c.opts.krylov_s ||
        o->mg_fused != c.opts.mg_fused || o->mg_first2 != c.opts.mg_first2)
        drop_graphs(c);
    c.opts = *o;
    return RBFIB_OK;
}

long long rbfib_state_size(const rbfib_ctx *ctx) { return ctx ? ctx->c.L : 0; }

int rbfib_layout(const rbfib_ctx *ctx, long long *out) {
    if (!ctx || !out) return RBFIB_EINVAL;
    const Ctx &c = ctx->c;
    for (int r = 0; r < c.nrep; ++r) {
        const RepDev &R = c.reps[r];
        out[4 * r + 0] = R.off;
        out[4 * r + 1] = R.off + 3 * R.N;
        out[4 * r + 2] = R.off + 4 * R.N;
        out[4 * r + 3] = R.off + 4 * R.N + 3LL * R.nm;
    }
    return RBFIB_OK;
}

__global__ void k_perm_local(const int *perm, const int *marker_body, const int *body_off_rep_m0, int nm, int *out) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nm) return;
    int m = perm[t];
    out[t] = m - body_off_rep_m0[marker_body[m]];
}

// Orders the library stream after the caller's stream on entry and the caller's
// stream after the library stream on exit.
struct Session {
    Ctx &c;
    explicit Session(Ctx &c_) : c(c_) {
        HIP_OK(hipEventRecord(c.ev_in, c.user_stream));
        HIP_OK(hipStreamWaitEvent(c.stream, c.ev_in, 0));
    }
    ~Session() {
        (void)hipEventRecord(c.ev_out, c.stream);
        (void)hipStreamWaitEvent(c.user_stream, c.ev_out, 0);
    }
};

int rbfib_markers(rbfib_ctx *ctx, const double *q, const double *theta, double *r, int *tile, int *perm) {
    if (!ctx || (ctx->c.nb > 0 && (!q || !theta))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    MarkerSet &ms = c.ms[0];
    const int st = build_markers(c, ms, q, theta, false);
    if (st != RBFIB_OK) return st;
    if (r && c.nm) HIP_OK(hipMemcpyAsync(r, ms.r, sizeof(double) * 3 * c.nm, hipMemcpyDeviceToDevice, c.stream));
    if (tile && c.nm) HIP_OK(hipMemcpyAsync(tile, ms.tile, sizeof(int) * c.nm, hipMemcpyDeviceToDevice, c.stream));
    if (perm && c.nm) {
        // replica-local ids: subtract each replica's first marker
        std::vector<int> m0(c.nb);
        for (int p = 0; p < c.nb; ++p) {
            int rr = 0;
            while (rr + 1 < c.nrep && c.reps[rr + 1].b0 <= p) ++rr;
            m0[p] = c.reps[rr].m0;
        }
        int *d_m0 = dalloc<int>(c.nb);
        HIP_OK(hipMemcpyAsync(d_m0, m0.data(), sizeof(int) * c.nb, hipMemcpyHostToDevice, c.stream));
        hipLaunchKernelGGL(k_perm_local, dim3((c.nm + 255) / 256), dim3(256), 0, c.stream, ms.perm, c.d_marker_body,
                           d_m0, c.nm, perm);
        HIP_OK(hipStreamSynchronize(c.stream));
        (void)hipFree(d_m0);
    }
    return RBFIB_OK;
    GUARD_END
}

int rbfib_apply_saddle(rbfib_ctx *ctx, const double *q, const double *theta, const double *x, double *y) {
    if (!ctx || !x || !y || x == y || (ctx->c.nb > 0 && (!q || !theta))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    const int st = build_markers(c, c.ms[0], q, theta, false);
    if (st != RBFIB_OK) return st;
    apply_op(c, c.ms[0], x, y, false);
    return RBFIB_OK;
    GUARD_END
}

int rbfib_precondition(rbfib_ctx *ctx, const double *q, const double *theta, const double *r, double *z) {
    if (!ctx || !r || !z || r == z || (ctx->c.nb > 0 && (!q || !theta))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    const int st = build_markers(c, c.ms[0], q, theta, false);
    if (st != RBFIB_OK) return st;
    precond(c, c.ms[0], stage_theta(c, theta), r, z, false);
    return RBFIB_OK;
    GUARD_END
}

int rbfib_solve_mobility(rbfib_ctx *ctx, const double *q, const double *theta, const double *FT, const double *slip,
                         int include_bc, double *U, double *x_out, rbfib_info *info) {
    if (!ctx || (ctx->c.nb > 0 && (!q || !theta || !FT))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    MarkerSet &ms = c.ms[0];
    int st = build_markers(c, ms, q, theta, true);
    if (st != RBFIB_OK) {
        if (info) for (int r = 0; r < c.nrep; ++r) info[r] = rbfib_info{0, 0.0, st};
        return st;
    }
    const double *th = stage_theta(c, theta);
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs(c, FT, slip, c.rhs);
    if (include_bc) add_boundary_terms(c, ms, c.rhs);
    std::vector<rbfib_info> inf;
    fgmres(c, ms, th, c.rhs, false, inf);
    if (U) launch_copy_U(c, c.xsol, U, 1.0);
    if (x_out) HIP_OK(hipMemcpyAsync(x_out, c.xsol, sizeof(double) * c.L, hipMemcpyDeviceToDevice, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    if (info) for (int r = 0; r < c.nrep; ++r) info[r] = inf[r];
    return first_bad(inf);
    GUARD_END
}

int rbfib_fluctuating_stress(rbfib_ctx *ctx, double kT, double dt, uint64_t seed, uint64_t step, double *f) {
    if (!ctx || !f || !(dt > 0.0) || kT < 0.0) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    launch_zero(c, f, nullptr);
    launch_noise(c, kT, dt, seed, step, f, false);
    return RBFIB_OK;
    GUARD_END
}

int rbfib_sem_step(rbfib_ctx *ctx, double *q, double *theta, const double *FT, const double *slip, double kT, double dt,
                   uint64_t seed, uint64_t step, double *U, rbfib_info *info) {
    if (!ctx || !(dt > 0.0) || !(kT >= 0.0) || (ctx->c.nb > 0 && (!q || !theta))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    std::vector<rbfib_info> inf;
    int code = sem_step(c, q, theta, FT, slip, kT, dt, seed, step, U, inf);
    HIP_OK(hipStreamSynchronize(c.stream));
    if (info) for (int r = 0; r < c.nrep; ++r) info[r] = inf[r];
    return code;
    GUARD_END
}

int rbfib_body_forces(rbfib_ctx *ctx, const double *q, const double *theta, const rbfib_potential *pot, double *FT) {
    if (!ctx || !pot || (ctx->c.nb > 0 && (!q || !theta || !FT))) return RBFIB_EINVAL;
    if (!(pot->b > 0.0) || !std::isfinite(pot->b) || !std::isfinite(pot->phi0) || !std::isfinite(pot->d) ||
        !std::isfinite(pot->fconst[0]) || !std::isfinite(pot->fconst[1]) || !std::isfinite(pot->fconst[2]))
        return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    launch_body_forces(c, q, theta, pot->phi0, pot->d, pot->b, pot->fconst, FT);
    HIP_OK(hipGetLastError());
    return RBFIB_OK;
    GUARD_END
}

int rbfib_sem_rk2_predict(rbfib_ctx *ctx, const double *q, const double *theta, const double *FT, const double *slip,
                          double kT, double dt, double alpha, uint64_t seed, uint64_t step, double *q_pred,
                          double *theta_pred, rbfib_info *info) {
    if (!ctx || !(dt > 0.0) || !(kT >= 0.0) || !(alpha > 0.0 && alpha <= 1.0) ||
        (ctx->c.nb > 0 && (!q || !theta || !FT || !q_pred || !theta_pred)))
        return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    c.trap_ready = false;
    const size_t nb = (size_t)c.nb;
    // configuration Q^n must be valid (the whole batch stops otherwise, as in rbfib_sem_step)
    const int st0 = build_markers(c, c.ms[0], q, theta, true);
    if (st0 != RBFIB_OK) {
        if (info)
            for (int r = 0; r < c.nrep; ++r)
                info[r] = rbfib_info{0, 0.0, c.h_flags[r] ? ((c.h_flags[r] & 8) ? RBFIB_EINVAL : RBFIB_EREJECT) : RBFIB_OK};
        return st0;
    }
    if (nb > 0) {
        HIP_OK(hipMemcpyAsync(c.trap_q0, q, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_th0, theta, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_q, q, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_th, theta, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
    }
    // Algorithm 1 at Q^n on the copies: U^n, and the Euler-Maruyama update Q* committed into them
    std::vector<rbfib_info> out, inf;
    const int code = sem_step(c, c.trap_q, c.trap_th, FT, slip, kT, dt, seed, step, c.trap_U, out);
    if (code != RBFIB_OK && code != RBFIB_EREJECT && code != RBFIB_ENOCONV) {
        if (info) for (int r = 0; r < c.nrep; ++r) info[r] = out[r];
        return code;
    }
    // deterministic velocity at Q^n (markers and orientations of Q^n are still staged)
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs(c, FT, slip, c.rhs);
    add_boundary_terms(c, c.ms[0], c.rhs);
    fgmres(c, c.ms[0], c.theta_int, c.rhs, false, inf);
    launch_copy_U(c, c.xsol, c.trap_U + 6 * nb, 1.0);
    if (alpha != 1.0 && nb > 0) {
        // the predictor moves Q^n by alpha dt U^n (the Euler-Maruyama update is alpha = 1);
        // replicas already rejected keep Q^n, others are rejected if Q* leaves the domain
        HIP_OK(hipMemcpyAsync(c.trap_q, c.trap_q0, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_th, c.trap_th0, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
        launch_rk2_update(c, c.trap_q0, c.trap_th0, c.trap_U, nullptr, nullptr, 0.0, alpha * dt, nullptr);
        clear_flags(c);
        launch_markers(c, c.ms[3], c.q_buf[2], c.th_buf[2]);
        HIP_OK(hipMemcpyAsync(c.h_flags, c.d_flags, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
        HIP_OK(hipStreamSynchronize(c.stream));
        for (int r = 0; r < c.nrep; ++r) {
            if (out[r].status != RBFIB_OK) c.h_flags[r] |= 4;
            else if (c.h_flags[r] & 3) out[r].status = RBFIB_EREJECT;
        }
        HIP_OK(hipMemcpyAsync(c.d_flags, c.h_flags, sizeof(int) * c.nrep, hipMemcpyHostToDevice, c.stream));
        launch_commit_positions(c, c.trap_q, c.trap_th);
    }
    if (nb > 0) {
        HIP_OK(hipMemcpyAsync(q_pred, c.trap_q, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(theta_pred, c.trap_th, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
    }
    HIP_OK(hipStreamSynchronize(c.stream));
    c.trap_status.assign(c.nrep, RBFIB_OK);
    int ret = RBFIB_OK;
    for (int r = 0; r < c.nrep; ++r) {
        out[r].iters += inf[r].iters;
        if (out[r].status == RBFIB_OK && inf[r].status != RBFIB_OK) out[r].status = inf[r].status;
        c.trap_status[r] = out[r].status;
        if (out[r].status != RBFIB_OK && ret == RBFIB_OK) ret = out[r].status;
    }
    if (info) for (int r = 0; r < c.nrep; ++r) info[r] = out[r];
    c.trap_dt = dt;
    c.trap_alpha = alpha;
    c.trap_ready = true;
    return ret;
    GUARD_END
}

int rbfib_sem_rk2_correct(rbfib_ctx *ctx, double *q, double *theta, const double *FT_pred, const double *slip_pred,
                          double *U, rbfib_info *info) {
    if (!ctx || !ctx->c.trap_ready || (ctx->c.nb > 0 && (!q || !theta || !FT_pred))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    c.trap_ready = false;
    const size_t nb = (size_t)c.nb;
    std::vector<rbfib_info> out(c.nrep, rbfib_info{0, 0.0, RBFIB_OK}), inf;
    // deterministic velocity at the predictor
    const int st = build_markers(c, c.ms[0], c.trap_q, c.trap_th, false);
    if (st != RBFIB_OK) return st;
    const double *th = stage_theta(c, c.trap_th);
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs(c, FT_pred, slip_pred, c.rhs);
    add_boundary_terms(c, c.ms[0], c.rhs);
    fgmres(c, c.ms[0], th, c.rhs, false, inf);
    launch_copy_U(c, c.xsol, c.trap_U + 12 * nb, 1.0);
    // corrector from Q^n, then the rejection test on Q^{n+1}
    launch_rk2_update(c, c.trap_q0, c.trap_th0, c.trap_U, c.trap_U + 6 * nb, c.trap_U + 12 * nb,
                      0.5 / c.trap_alpha, c.trap_dt, c.Fp);
    clear_flags(c);
    launch_markers(c, c.ms[3], c.q_buf[2], c.th_buf[2]);
    launch_body_distance(c, c.opts.min_body_dist);
    HIP_OK(hipMemcpyAsync(c.h_flags, c.d_flags, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    for (int r = 0; r < c.nrep; ++r) {
        out[r] = inf[r];
        // replicas whose predictor step was rejected or failed, or whose solve failed, keep Q^n
        if (c.trap_status[r] != RBFIB_OK || inf[r].status != RBFIB_OK) c.h_flags[r] |= 4;
    }
    HIP_OK(hipMemcpyAsync(c.d_flags, c.h_flags, sizeof(int) * c.nrep, hipMemcpyHostToDevice, c.stream));
    launch_commit_positions(c, q, theta);
    if (U && nb > 0) HIP_OK(hipMemcpyAsync(U, c.Fp, sizeof(double) * 6 * nb, hipMemcpyDeviceToDevice, c.stream));
    read_flags(c);
    int ret = RBFIB_OK;
    for (int r = 0; r < c.nrep; ++r) {
        if (c.trap_status[r] != RBFIB_OK) out[r].status = c.trap_status[r];
        else if (out[r].status == RBFIB_OK && (c.h_flags[r] & 3)) out[r].status = RBFIB_EREJECT;
        if (out[r].status != RBFIB_OK && ret == RBFIB_OK) ret = out[r].status;
    }
    if (info) for (int r = 0; r < c.nrep; ++r) info[r] = out[r];
    return ret;
    GUARD_END
}

int rbfib_sem_ab2_step(rbfib_ctx *ctx, double *q, double *theta, const double *FT, const double *slip, double kT,
                       double dt, uint64_t seed, uint64_t step, double *U_det_prev, int have_prev, double *U,
                       rbfib_info *info) {
    if (!ctx || !(dt > 0.0) || !(kT >= 0.0) || (have_prev != 0 && have_prev != 1) ||
        (ctx->c.nb > 0 && (!q || !theta || !FT || !U_det_prev)))
        return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    c.trap_ready = false;                       // the stage buffers are reused here
    const size_t nb = (size_t)c.nb;
    const int st0 = build_markers(c, c.ms[0], q, theta, true);
    if (st0 != RBFIB_OK) {
        if (info)
            for (int r = 0; r < c.nrep; ++r)
                info[r] = rbfib_info{0, 0.0, c.h_flags[r] ? ((c.h_flags[r] & 8) ? RBFIB_EINVAL : RBFIB_EREJECT) : RBFIB_OK};
        return st0;
    }
    if (nb > 0) {
        HIP_OK(hipMemcpyAsync(c.trap_q0, q, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_th0, theta, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_q, q, sizeof(double) * 3 * nb, hipMemcpyDeviceToDevice, c.stream));
        HIP_OK(hipMemcpyAsync(c.trap_th, theta, sizeof(double) * 4 * nb, hipMemcpyDeviceToDevice, c.stream));
    }
    // Algorithm 1 at Q^n (on copies) for U^n, then the deterministic velocity at Q^n
    std::vector<rbfib_info> out, inf;
    const int code = sem_step(c, c.trap_q, c.trap_th, FT, slip, kT, dt, seed, step, c.trap_U, out);
    if (code != RBFIB_OK && code != RBFIB_EREJECT && code != RBFIB_ENOCONV) {
        if (info) for (int r = 0; r < c.nrep; ++r) info[r] = out[r];
        return code;
    }
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs(c, FT, slip, c.rhs);
    add_boundary_terms(c, c.ms[0], c.rhs);
    fgmres(c, c.ms[0], c.theta_int, c.rhs, false, inf);
    double *Ud = c.trap_U + 6 * nb;
    launch_copy_U(c, c.xsol, Ud, 1.0);
    // U_c = U^n + (U_det^n - U_det^{n-1}) / 2 from Q^n, then the rejection test on Q^{n+1}
    launch_rk2_update(c, c.trap_q0, c.trap_th0, c.trap_U, have_prev ? U_det_prev : Ud, Ud, 0.5, dt, c.Fp);
    clear_flags(c);
    launch_markers(c, c.ms[3], c.q_buf[2], c.th_buf[2]);
    launch_body_distance(c, c.opts.min_body_dist);
    HIP_OK(hipMemcpyAsync(c.h_flags, c.d_flags, sizeof(int) * c.nrep, hipMemcpyDeviceToHost, c.stream));
    HIP_OK(hipStreamSynchronize(c.stream));
    for (int r = 0; r < c.nrep; ++r) {
        out[r].iters += inf[r].iters;
        if (out[r].status == RBFIB_OK && inf[r].status != RBFIB_OK) out[r].status = inf[r].status;
        if (out[r].status != RBFIB_OK) c.h_flags[r] |= 4;
    }
    HIP_OK(hipMemcpyAsync(c.d_flags, c.h_flags, sizeof(int) * c.nrep, hipMemcpyHostToDevice, c.stream));
    launch_commit_positions(c, q, theta);
    if (nb > 0) {
        HIP_OK(hipMemcpyAsync(U_det_prev, Ud, sizeof(double) * 6 * nb, hipMemcpyDeviceToDevice, c.stream));
        if (U) HIP_OK(hipMemcpyAsync(U, c.Fp, sizeof(double) * 6 * nb, hipMemcpyDeviceToDevice, c.stream));
    }
    read_flags(c);
    int ret = RBFIB_OK;
    for (int r = 0; r < c.nrep; ++r) {
        if (out[r].status == RBFIB_OK && (c.h_flags[r] & 3)) out[r].status = RBFIB_EREJECT;
        if (out[r].status != RBFIB_OK && ret == RBFIB_OK) ret = out[r].status;
    }
    if (info) for (int r = 0; r < c.nrep; ++r) info[r] = out[r];
    return ret;
    GUARD_END
}

int rbfib_mobility_vjp(rbfib_ctx *ctx, const double *q, const double *theta, const double *FT, const double *Ubar,
                       double *dFT, double *dq, double *dphi, double *dtheta, rbfib_info *info) {
    if (!ctx || (ctx->c.nb > 0 && (!q || !theta || !FT || !Ubar))) return RBFIB_EINVAL;
    GUARD_BEGIN
    Ctx &c = ctx->c;
    Session s(c);
    int st = build_markers(c, c.ms[0], q, theta, true);
    if (st != RBFIB_OK) {
        if (info) for (int r = 0; r < c.nrep; ++r) info[r] = rbfib_info{0, 0.0, st};
        return st;
    }
    const double *th = stage_theta(c, theta);
    std::vector<rbfib_info> fwd, adj;
    // forward solve (the Krylov basis is recomputed, not stored)
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs(c, FT, nullptr, c.rhs);
    fgmres(c, c.ms[0], th, c.rhs, false, fwd);
    HIP_OK(hipMemcpyAsync(c.xR, c.xsol, sizeof(double) * c.L, hipMemcpyDeviceToDevice, c.stream));
    // adjoint solve with the same operator
    launch_zero(c, c.rhs, nullptr);
    launch_set_rhs_adjoint(c, Ubar, c.rhs);
    fgmres(c, c.ms[0], th, c.rhs, false, adj);
    launch_body_grad(c, c.xR, c.xsol, theta, dFT, dq, dphi, dtheta);
    HIP_OK(hipStreamSynchronize(c.stream));
    int ret = RBFIB_OK;
    for (int r = 0; r < c.nrep; ++r) {
        rbfib_info i{fwd[r].iters + adj[r].iters, std::max(fwd[r].rel_residual, adj[r].rel_residual),
                     fwd[r].status != RBFIB_OK ? fwd[r].status : adj[r].status};
        if (info) info[r] = i;
        if (i.status != RBFIB_OK && ret == RBFIB_OK) ret = i.status;
    }
    return ret;
    GUARD_END
}

int rbfib_launch_geometry(const rbfib_ctx *ctx, int *out) {
    if (!ctx || !out) return RBFIB_EINVAL;
    const Ctx &c = ctx->c;
    out[0] = c.tune.krylov_chunk;
    out[1] = c.tune.spread_grid;
    out[2] = c.tune.spread_p;
    out[3] = c.mg_npt;
    out[4] = c.apply_kc;
    return RBFIB_OK;
}

int rbfib_enable_timing(rbfib_ctx *ctx, int on) {
    if (!ctx) return RBFIB_EINVAL;
    ctx->c.timing.on = on != 0;
    for (int k = 0; k < RB_NTIMING; ++k) {
        ctx->c.timing.total_ms[k] = 0; ctx->c.timing.bytes[k] = 0; ctx->c.timing.launches[k] = 0; ctx->c.timing.used[k] = 0;
    }
    return RBFIB_OK;
}

int rbfib_kernel_stats(rbfib_ctx *ctx, int which, double *avg_ms, double *bytes_per_launch, long long *launches) {
    if (!ctx || which < 0 || which >= RB_NTIMING) return RBFIB_EINVAL;
    Ctx &c = ctx->c;
    long long n = c.timing.launches[which];
    if (avg_ms) *avg_ms = n ? c.timing.total_ms[which] / n : 0.0;
    if (launches) *launches = n;
    if (bytes_per_launch) *bytes_per_launch = n ? c.timing.bytes[which] / n : 0.0;
    return RBFIB_OK;
}

}  // extern "C"

// Fused multigrid level kernels (two damped-Jacobi sweeps per level).
//
// k_mg_down (one workgroup per coarse tile of level l+1): stages b of level l on
// the tile's fine region plus a two-point halo in LDS, takes the first sweep from
// zero (x1 = omega D^-1 b), the second sweep, writes the smoothed x of the fine
// points the tile owns, forms the residual and restricts it to the coarse tile:
// one read of b, one write of x and of the coarse right-hand side, instead of
// three launches and four passes.
//
// k_mg_up (one workgroup per fine tile of level l): x + P x_coarse on the tile
// plus a two-point halo, then two sweeps in LDS, one write.
//
// The operator, boundary rules, transfer weights and damping are those of the
// unfused kernels in grid.hip (face-normal wall faces Dirichlet, odd ghosts for
// tangential velocity, even ghosts for pressure, periodic wrap), applied in
// global coordinates so that halo points outside a wall are never read.
#include "common.h"

namespace rb {

template <typename T> struct TileShape;
template <> struct TileShape<float> {
    static constexpr int CX = MGD32_X, CY = MGD32_Y, CZ = MGD32_Z, FX = MGU32_X, FY = MGU32_Y, FZ = MGU32_Z;
};
template <> struct TileShape<double> {
    static constexpr int CX = MGD64_X, CY = MGD64_Y, CZ = MGD64_Z, FX = MGU64_X, FY = MGU64_Y, FZ = MGU64_Z;
};

__device__ __forceinline__ bool is_pinned(int comp, const int g[3], const int bc[3]) {
    return comp < 3 && bc[comp] == RBFIB_WALL && g[comp] == 0;
}

// global coordinate of box position (lo + l) along an axis; false when outside a wall
__device__ __forceinline__ bool box_coord(int lo, int l, int n, int bc, int &g) {
    g = lo + l;
    if (bc == RBFIB_PERIODIC) {
        g %= n;
        if (g < 0) g += n;
        return true;
    }
    return g >= 0 && g < n;
}

template <typename T>
__device__ __forceinline__ T diag_at(int comp, const int g[3], const int n[3], const int bc[3], const double ih2[3]) {
    T dg = (T)0;
    for (int a = 0; a < 3; ++a) {
        T da = (T)-2;
        if (bc[a] == RBFIB_WALL && a != comp) {
            T gg = (comp == 3) ? (T)1 : (T)-1;
            if (g[a] == 0) da += gg;
            if (g[a] == n[a] - 1) da += gg;
        }
        dg += da * (T)ih2[a];
    }
    return dg;
}

// sum_a (u(+a) - 2u + u(-a)) ih2[a] at box point li (interior of the box), with
// the boundary rule and the association of the unfused stencil.
template <typename T>
__device__ __forceinline__ T box_nbr(const T *A, int li, int stride, int d, T self, int q, int n, int bc, int a,
                                     int comp) {
    if (bc == RBFIB_PERIODIC) return A[li + d * stride];
    if (a == comp) return (q <= 0 || q >= n) ? (T)0 : A[li + d * stride];
    if (q < 0 || q >= n) return (comp == 3) ? self : -self;
    return A[li + d * stride];
}

template <typename T>
__device__ __forceinline__ T lap_box(const T *A, int li, const int S[3], const int g[3], int comp, const int n[3],
                                     const int bc[3], const double ih2[3]) {
    T self = A[li];
    T acc = (T)0;
    int stride = 1;
    for (int a = 0; a < 3; ++a) {
        T up = box_nbr<T>(A, li, stride, +1, self, g[a] + 1, n[a], bc[a], a, comp);
        T um = box_nbr<T>(A, li, stride, -1, self, g[a] - 1, n[a], bc[a], a, comp);
        acc += (up - (T)2 * self + um) * (T)ih2[a];
        stride *= S[a];
    }
    return acc;
}

// ------------------------------------------------------------------ down
template <typename T>
__global__ __launch_bounds__(256) void k_mg_down(const RepDev *reps, const LevDev *levs, const BlockEnt *tab,
                                                  int lev, int c0, const T *bpool, T *__restrict__ xpool, T *bcpool,
                                                  double omega, const int *__restrict__ mask) {
    constexpr int CX = TileShape<T>::CX, CY = TileShape<T>::CY, CZ = TileShape<T>::CZ;
    // box extent: 2 C + 5 along the face-normal axis of the component, 2 C + 4 along the others
    constexpr int B0 = (2 * CX + 5) * (2 * CY + 4) * (2 * CZ + 4);
    constexpr int B1 = (2 * CX + 4) * (2 * CY + 5) * (2 * CZ + 4);
    constexpr int B2 = (2 * CX + 4) * (2 * CY + 4) * (2 * CZ + 5);
    constexpr int MAXB = B0 > B1 ? (B0 > B2 ? B0 : B2) : (B1 > B2 ? B1 : B2);
    __shared__ T B[MAXB];
    __shared__ T X1[MAXB];
    __shared__ T X2[MAXB];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    const int TC[3] = {CX, CY, CZ};
    int ntc[3], tc[3], cl[3], ce[3], rlo[3], rhi[3], blo[3], S[3];
    for (int a = 0; a < 3; ++a) ntc[a] = (C.n[a] + TC[a] - 1) / TC[a];
    long long t = be.start;
    tc[0] = (int)(t % ntc[0]); t /= ntc[0];
    tc[1] = (int)(t % ntc[1]); tc[2] = (int)(t / ntc[1]);
    bool crs[3];
    for (int a = 0; a < 3; ++a) {
        crs[a] = F.n[a] != C.n[a];
        cl[a] = tc[a] * TC[a];
        ce[a] = min(TC[a], C.n[a] - cl[a]);
        if (crs[a]) {
            rlo[a] = 2 * cl[a] - (a == comp ? 1 : 0);
            rhi[a] = 2 * (cl[a] + ce[a]) - 1;
        } else {
            rlo[a] = cl[a];
            rhi[a] = cl[a] + ce[a] - 1;
        }
        blo[a] = rlo[a] - 2;
        S[a] = rhi[a] - rlo[a] + 5;
    }
    const int nbox = S[0] * S[1] * S[2];
    const T *b = bpool + F.off + comp * F.N;
    T *x = xpool + F.off + comp * F.N;
    T *bc = bcpool + C.off + comp * C.N;
    const long long n01 = (long long)F.n[0] * F.n[1];
    // phase 1: b on the box, x1 = omega D^-1 b
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        T bv = (T)0, x1 = (T)0;
        if (in && !is_pinned(comp, g, R.bc)) {
            bv = b[g[0] + (long long)F.n[0] * g[1] + n01 * g[2]];
            x1 = (T)omega * bv / (s * diag_at<T>(comp, g, F.n, R.bc, F.inv_h2));
        }
        B[li] = bv;
        X1[li] = x1;
    }
    __syncthreads();
    // phase 2: second sweep on the region plus one halo point
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        if (l[0] < 1 || l[0] > S[0] - 2 || l[1] < 1 || l[1] > S[1] - 2 || l[2] < 1 || l[2] > S[2] - 2) continue;
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        T x2 = (T)0;
        if (in && !is_pinned(comp, g, R.bc)) {
            T dg = diag_at<T>(comp, g, F.n, R.bc, F.inv_h2);
            T lap = lap_box<T>(X1, li, S, g, comp, F.n, R.bc, F.inv_h2);
            x2 = X1[li] + (T)omega * (B[li] - s * lap) / (s * dg);
        }
        X2[li] = x2;
    }
    __syncthreads();
    // phase 3: write the owned fine points; residual on the restriction region
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        if (l[0] < 2 || l[0] > S[0] - 3 || l[1] < 2 || l[1] > S[1] - 3 || l[2] < 2 || l[2] > S[2] - 3) continue;
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        T r = (T)0;
        if (in) {
            bool own = true;
            for (int a = 0; a < 3; ++a) {
                int gl = blo[a] + l[a];          // unwrapped
                int olo = crs[a] ? 2 * cl[a] : cl[a];
                int ohi = crs[a] ? 2 * (cl[a] + ce[a]) - 1 : cl[a] + ce[a] - 1;
                own &= (gl >= olo && gl <= ohi);
            }
            long long gi = g[0] + (long long)F.n[0] * g[1] + n01 * g[2];
            if (own) x[gi] = X2[li];
            if (!is_pinned(comp, g, R.bc)) r = B[li] - s * lap_box<T>(X2, li, S, g, comp, F.n, R.bc, F.inv_h2);
        }
        X1[li] = r;      // X1 no longer needed: residual on the region
    }
    __syncthreads();
    // phase 4: restriction to the coarse tile
    const int nct = ce[0] * ce[1] * ce[2];
    const long long c01 = (long long)C.n[0] * C.n[1];
    for (int k = threadIdx.x; k < nct; k += blockDim.x) {
        int ci[3] = {cl[0] + k % ce[0], cl[1] + (k / ce[0]) % ce[1], cl[2] + k / (ce[0] * ce[1])};
        long long cgi = ci[0] + (long long)C.n[0] * ci[1] + c01 * ci[2];
        if (is_pinned(comp, ci, R.bc)) { bc[cgi] = (T)0; continue; }
        // per axis: first box index of the fine points, their count, and whether
        // the axis is the face-normal one (weights 1/4, 1/2, 1/4) or a cell axis (1/2, 1/2)
        int fb[3], fc[3];
        bool face[3];
        for (int a = 0; a < 3; ++a) {
            face[a] = crs[a] && a == comp;
            fc[a] = !crs[a] ? 1 : (face[a] ? 3 : 2);
            fb[a] = (crs[a] ? 2 * ci[a] - (face[a] ? 1 : 0) : ci[a]) - blo[a];
        }
        T acc = (T)0;
        for (int kk = 0; kk < fc[2]; ++kk) {
            const T wz = restrict_weight<T>(crs[2], face[2], kk);
            for (int jj = 0; jj < fc[1]; ++jj) {
                const T wy = restrict_weight<T>(crs[1], face[1], jj);
                for (int ii = 0; ii < fc[0]; ++ii) {
                    const T wx = restrict_weight<T>(crs[0], face[0], ii);
                    acc += wx * wy * wz * X1[fb[0] + ii + S[0] * (fb[1] + jj + S[1] * (fb[2] + kk))];
                }
            }
        }
        bc[cgi] = acc;
    }
}

// ------------------------------------------------------------------ up
template <typename T>
__global__ __launch_bounds__(256) void k_mg_up(const RepDev *reps, const LevDev *levs, const BlockEnt *tab, int lev,
                                                int c0, const T *__restrict__ bpool, const T *__restrict__ xinpool,
                                                const T *__restrict__ xcpool, T *__restrict__ xoutpool, double omega,
                                                const int *__restrict__ mask) {
    constexpr int FX = TileShape<T>::FX, FY = TileShape<T>::FY, FZ = TileShape<T>::FZ;
    constexpr int MAXB = (FX + 4) * (FY + 4) * (FZ + 4);
    __shared__ T XP[MAXB];
    __shared__ T XS[MAXB];
    BlockEnt be = tab[blockIdx.x];
    if (mask && !mask[be.rep]) return;
    const int comp = c0 + blockIdx.y;
    const RepDev &R = reps[be.rep];
    const LevDev &F = levs[be.rep * RB_MAXLEV + lev];
    const LevDev &C = levs[be.rep * RB_MAXLEV + lev + 1];
    const T s = (comp < 3) ? (T)(-R.eta) : (T)-1;
    const int TF[3] = {FX, FY, FZ};
    int ntf[3], tl[3], te[3], blo[3], S[3];
    for (int a = 0; a < 3; ++a) ntf[a] = (F.n[a] + TF[a] - 1) / TF[a];
    long long t = be.start;
    int tcoord[3];
    tcoord[0] = (int)(t % ntf[0]); t /= ntf[0];
    tcoord[1] = (int)(t % ntf[1]); tcoord[2] = (int)(t / ntf[1]);
    for (int a = 0; a < 3; ++a) {
        tl[a] = tcoord[a] * TF[a];
        te[a] = min(TF[a], F.n[a] - tl[a]);
        blo[a] = tl[a] - 2;
        S[a] = te[a] + 4;
    }
    const int nbox = S[0] * S[1] * S[2];
    const T *b = bpool + F.off + comp * F.N;
    const T *xin = xinpool + F.off + comp * F.N;
    T *x = xoutpool + F.off + comp * F.N;
    const T *xc = xcpool + C.off + comp * C.N;
    const long long n01 = (long long)F.n[0] * F.n[1];
    // phase 1: x + P x_c on the box (x read from the down pass, never from the output)
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        T v = (T)0;
        if (in && !is_pinned(comp, g, R.bc))
            v = xin[g[0] + (long long)F.n[0] * g[1] + n01 * g[2]] + prolong_at<T>(R, F, C, comp, g, xc);
        XP[li] = v;
    }
    __syncthreads();
    // phase 2: first post-smoothing sweep on the tile plus one halo point
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        if (l[0] < 1 || l[0] > S[0] - 2 || l[1] < 1 || l[1] > S[1] - 2 || l[2] < 1 || l[2] > S[2] - 2) continue;
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        T v = (T)0;
        if (in && !is_pinned(comp, g, R.bc)) {
            T dg = diag_at<T>(comp, g, F.n, R.bc, F.inv_h2);
            T lap = lap_box<T>(XP, li, S, g, comp, F.n, R.bc, F.inv_h2);
            T bv = b[g[0] + (long long)F.n[0] * g[1] + n01 * g[2]];
            v = XP[li] + (T)omega * (bv - s * lap) / (s * dg);
        }
        XS[li] = v;
    }
    __syncthreads();
    // phase 3: second sweep on the tile, written back
    for (int li = threadIdx.x; li < nbox; li += blockDim.x) {
        int l[3] = {li % S[0], (li / S[0]) % S[1], li / (S[0] * S[1])};
        if (l[0] < 2 || l[0] > S[0] - 3 || l[1] < 2 || l[1] > S[1] - 3 || l[2] < 2 || l[2] > S[2] - 3) continue;
        int g[3];
        bool in = true;
        for (int a = 0; a < 3; ++a) in &= box_coord(blo[a], l[a], F.n[a], R.bc[a], g[a]);
        if (!in) continue;
        long long gi = g[0] + (long long)F.n[0] * g[1] + n01 * g[2];
        if (is_pinned(comp, g, R.bc)) { x[gi] = (T)0; continue; }
        T dg = diag_at<T>(comp, g, F.n, R.bc, F.inv_h2);
        T lap = lap_box<T>(XS, li, S, g, comp, F.n, R.bc, F.inv_h2);
        x[gi] = XS[li] + (T)omega * (b[gi] - s * lap) / (s * dg);
    }
}

template <typename T>
void launch_mg_down(Ctx &c, int lev, int c0, int nc, const T *b, T *x) {
    int n = c.n_tab_down[lev];
    if (n == 0) return;
    hipLaunchKernelGGL(k_mg_down<T>, dim3(n, nc), dim3(256), 0, c.stream, c.d_reps, c.d_levs, c.d_tab_down[lev], lev,
                       c0, b, x, (T *)b, c.opts.mg_omega, c.mask);
    HIP_OK(hipGetLastError());
}

template <typename T>
void launch_mg_up(Ctx &c, int lev, int c0, int nc, const T *b, const T *xin, const T *xc, T *xout) {
    int n = c.n_tab_up[lev];
    if (n == 0) return;
    hipLaunchKernelGGL(k_mg_up<T>, dim3(n, nc), dim3(256), 0, c.stream, c.d_reps, c.d_levs, c.d_tab_up[lev], lev, c0,
                       b, xin, xc, xout, c.opts.mg_omega, c.mask);
    HIP_OK(hipGetLastError());
}

template void launch_mg_down<float>(Ctx &, int, int, int, const float *, float *);
template void launch_mg_down<double>(Ctx &, int, int, int, const double *, double *);
template void launch_mg_up<float>(Ctx &, int, int, int, const float *, const float *, const float *, float *);
template void launch_mg_up<double>(Ctx &, int, int, int, const double *, const double *, const double *, double *);

}  // namespace rb

// Allocation-free saddle-operator apply for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that forbid
// hipMalloc): one replica, y = A x exactly as rbfib_apply_saddle computes it, with
// every table the kernels need -- replica descriptor, body and marker maps, marker
// positions and cached kernel weights, tile bins, spreading pairs, scan partials and
// the block table of the stencil sweep -- in one file-scope device array of fixed
// size instead of a context's workspace.
//
// The array is a host-side stand-in in host code: its device address is taken once
// per device with hipGetSymbolAddress (on the first call on that device, with the
// device current) and only that address is ever passed to kernels.  Each device
// holds its own copy until the process ends.  Calls on one device share it: they are
// ordered on one stream, or race.
#include "common.h"

#include <algorithm>
#include <mutex>

namespace rb {

// Limits of the allocation-free apply (sizes beyond them are rejected with
// RBFIB_EINVAL before any work is enqueued).
#define RBNA_MAX_MARKERS 8192
#define RBNA_MAX_BODIES 2048
#define RBNA_MAX_BODY_MARKERS 1024        // k_body_apply stages 6 doubles per marker of a body in LDS
#define RBNA_MAX_CELLS (1LL << 23)
#define RBNA_MAX_TILES (1 << 17)
#define RBNA_MAX_PAIRS (27LL * RBNA_MAX_MARKERS)
#define RBNA_MAX_TAB (int)((RBNA_MAX_CELLS + 2 * RB_BLOCK - 1) / (2 * RB_BLOCK))

// Byte layout of the scratch array: sections in a fixed order, each 256-byte aligned.
struct NaLayout {
    size_t reps, marker_body, body_rep, body_off, tile_rep, rref, tab, flags, scan;
    size_t r, d, tile, perm, tile_count, tile_start, tile_fill, active, n_active;
    size_t pair_count, pair_start, pair_fill, pair_m, pair_tile, wc, ic;
    size_t total;
};

static constexpr size_t na_align(size_t v) { return (v + 255) & ~(size_t)255; }

static constexpr NaLayout na_layout() {
    NaLayout L{};
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t at = o; o = na_align(o + bytes); return at; };
    const size_t M = RBNA_MAX_MARKERS, B = RBNA_MAX_BODIES, T = RBNA_MAX_TILES;
    L.reps = take(sizeof(RepDev));
    L.marker_body = take(sizeof(int) * M);
    L.body_rep = take(sizeof(int) * B);
    L.body_off = take(sizeof(int) * (B + 1));
    L.tile_rep = take(sizeof(int) * T);
    L.rref = take(sizeof(double) * 3 * M);
    L.tab = take(sizeof(BlockEnt) * RBNA_MAX_TAB);
    L.flags = take(sizeof(int) * 4);
    L.scan = take(sizeof(int) * ((T + 1023) / 1024 + 1));
    L.r = take(sizeof(double) * 3 * M);
    L.d = take(sizeof(double) * 3 * M);
    L.tile = take(sizeof(int) * M);
    L.perm = take(sizeof(int) * M);
    L.tile_count = take(sizeof(int) * T);
    L.tile_start = take(sizeof(int) * T);
    L.tile_fill = take(sizeof(int) * T);
    L.active = take(sizeof(int) * T);
    L.n_active = take(sizeof(int));
    L.pair_count = take(sizeof(int) * T);
    L.pair_start = take(sizeof(int) * T);
    L.pair_fill = take(sizeof(int) * T);
    L.pair_m = take(sizeof(int) * RBNA_MAX_PAIRS);
    L.pair_tile = take(sizeof(int) * RBNA_MAX_PAIRS);
    L.wc = take(sizeof(double) * 36 * M);
    L.ic = take(sizeof(int) * 36 * M);
    L.total = o;
    return L;
}

static constexpr NaLayout NA = na_layout();

// The scratch array (about 10 MiB), one copy per device.
static __device__ __align__(256) unsigned char scratch[NA.total];

// Per-device address of `scratch`, taken once per device with that device current.
static std::mutex g_na_mutex;
static unsigned char *g_na_ptr[64] = {nullptr};

static unsigned char *scratch_address() {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw (int)RBFIB_EDEVICE;
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_na_ptr[dev] = static_cast<unsigned char *>(p);
    }
    return g_na_ptr[dev];
}

// Set-up kernel: replica descriptor, body and marker maps (from the uploaded
// marker offsets), tile -> replica map, the stencil block table (two cells per
// thread, as the apply's), and zeroed tile and pair counts and flags.  One pass over
// max(markers, tiles, table entries) threads.
__global__ void k_na_setup(RepDev rep, int nb, int nm, int ntiles, int ntab, RepDev *reps, int *marker_body,
                           int *body_rep, int *body_off, int *tile_rep, BlockEnt *tab, int *tile_count,
                           int *pair_count, int *flags, int *n_active) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        reps[0] = rep;
        for (int k = 0; k < 4; ++k) flags[k] = 0;
        *n_active = 0;
    }
    if (i < nb) {
        body_rep[i] = 0;
        for (int m = body_off[i]; m < body_off[i + 1]; ++m) marker_body[m] = i;
    }
    if (i < ntiles) {
        tile_rep[i] = 0;
        tile_count[i] = 0;
        pair_count[i] = 0;
    }
    if (i < ntab) tab[i] = BlockEnt{0, 2, (long long)i * 2 * RB_BLOCK};
}

static int apply_noalloc(const rbfib_grid *grid, const rbfib_bodies *bodies, const double *q, const double *theta,
                         const double *x, double *y, hipStream_t stream) {
    if (!grid || !bodies || !x || !y || x == y) return RBFIB_EINVAL;
    const rbfib_grid &g = *grid;
    const rbfib_bodies &bd = *bodies;
    int walls = 0, periodic = 0;
    for (int a = 0; a < 3; ++a) {
        if (g.n[a] < 4 || g.n[a] > (1 << 16)) return RBFIB_EINVAL;
        if (g.bc[a] != RBFIB_PERIODIC && g.bc[a] != RBFIB_WALL && g.bc[a] != RBFIB_SLIP) return RBFIB_EINVAL;
        walls += g.bc[a] == RBFIB_WALL;
        periodic += g.bc[a] == RBFIB_PERIODIC;
    }
    if ((walls == 0 && periodic > 0) || periodic == 3 || !(g.h > 0.0) || !(g.eta > 0.0)) return RBFIB_EINVAL;
    const long long N = (long long)g.n[0] * g.n[1] * g.n[2];
    const long long ntiles = (long long)((g.n[0] + 3) / 4) * ((g.n[1] + 3) / 4) * ((g.n[2] + 3) / 4);
    if (N > RBNA_MAX_CELLS || ntiles > RBNA_MAX_TILES) return RBFIB_EINVAL;
    if (bd.nb < 0 || bd.nm < 0 || bd.nb > RBNA_MAX_BODIES || bd.nm > RBNA_MAX_MARKERS) return RBFIB_EINVAL;
    if (bd.nb > 0 && (!bd.marker_offset || !bd.r_ref || !q || !theta)) return RBFIB_EINVAL;
    int max_body = 1;
    if (bd.nb > 0) {
        if (bd.marker_offset[0] != 0 || bd.marker_offset[bd.nb] != bd.nm) return RBFIB_EINVAL;
        for (int p = 0; p < bd.nb; ++p) {
            const int n = bd.marker_offset[p + 1] - bd.marker_offset[p];
            if (n <= 0 || n > RBNA_MAX_BODY_MARKERS) return RBFIB_EINVAL;
            max_body = std::max(max_body, n);
        }
    } else if (bd.nm != 0) {
        return RBFIB_EINVAL;
    }
    unsigned char *base = scratch_address();

    // a stack context whose device pointers all point into the scratch array
    Ctx c;
    c.stream = stream;
    c.nrep = 1;
    c.nb = bd.nb;
    c.nm = bd.nm;
    c.ntiles = (int)ntiles;
    c.max_body_nm = max_body;
    c.d_reps = reinterpret_cast<RepDev *>(base + NA.reps);
    c.d_marker_body = reinterpret_cast<int *>(base + NA.marker_body);
    c.d_body_rep = reinterpret_cast<int *>(base + NA.body_rep);
    c.d_body_off = reinterpret_cast<int *>(base + NA.body_off);
    c.d_tile_rep = reinterpret_cast<int *>(base + NA.tile_rep);
    c.d_rref = reinterpret_cast<double *>(base + NA.rref);
    c.d_tab_cells2 = reinterpret_cast<BlockEnt *>(base + NA.tab);
    c.n_tab_cells2 = (int)((N + 2 * RB_BLOCK - 1) / (2 * RB_BLOCK));
    c.d_flags = reinterpret_cast<int *>(base + NA.flags);
    c.d_scan = reinterpret_cast<int *>(base + NA.scan);
    MarkerSet &ms = c.ms[0];
    ms.r = reinterpret_cast<double *>(base + NA.r);
    ms.d = reinterpret_cast<double *>(base + NA.d);
    ms.tile = reinterpret_cast<int *>(base + NA.tile);
    ms.perm = reinterpret_cast<int *>(base + NA.perm);
    ms.tile_count = reinterpret_cast<int *>(base + NA.tile_count);
    ms.tile_start = reinterpret_cast<int *>(base + NA.tile_start);
    ms.tile_fill = reinterpret_cast<int *>(base + NA.tile_fill);
    ms.active = reinterpret_cast<int *>(base + NA.active);
    ms.n_active = reinterpret_cast<int *>(base + NA.n_active);
    ms.pair_count = reinterpret_cast<int *>(base + NA.pair_count);
    ms.pair_start = reinterpret_cast<int *>(base + NA.pair_start);
    ms.pair_fill = reinterpret_cast<int *>(base + NA.pair_fill);
    ms.pair_m = reinterpret_cast<int *>(base + NA.pair_m);
    ms.pair_tile = reinterpret_cast<int *>(base + NA.pair_tile);
    ms.wc = reinterpret_cast<double *>(base + NA.wc);
    ms.ic = reinterpret_cast<int *>(base + NA.ic);
    // spreading pairs: at most two tiles per axis, three on a periodic axis that ends
    // in a partial tile, never more than the axis has (as for a context)
    long long per = 1;
    for (int a = 0; a < 3; ++a) {
        const int tdim = (g.n[a] + RB_TILE - 1) / RB_TILE;
        const int b = (g.bc[a] == RBFIB_PERIODIC && g.n[a] % RB_TILE != 0) ? 3 : 2;
        per *= std::min(b, tdim);
    }
    ms.pair_cap = std::max(1LL, per * bd.nm);
    if (ms.pair_cap > RBNA_MAX_PAIRS) return RBFIB_EINVAL;

    RepDev R;
    rep_from_grid(R, g, bd.nb, bd.nm, 0, 0, 0, 0);
    // body offsets and body-frame marker offsets come from host memory
    if (bd.nb > 0) {
        HIP_OK(hipMemcpyAsync(c.d_body_off, bd.marker_offset, sizeof(int) * (bd.nb + 1), hipMemcpyHostToDevice,
                              stream));
        HIP_OK(hipMemcpyAsync(c.d_rref, bd.r_ref, sizeof(double) * 3 * bd.nm, hipMemcpyHostToDevice, stream));
    }
    const long long work = std::max({(long long)bd.nm, (long long)bd.nb, ntiles, (long long)c.n_tab_cells2, 1LL});
    hipLaunchKernelGGL(k_na_setup, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, stream, R, bd.nb, bd.nm,
                       c.ntiles, c.n_tab_cells2, c.d_reps, c.d_marker_body, c.d_body_rep, c.d_body_off,
                       c.d_tile_rep, c.d_tab_cells2, ms.tile_count, ms.pair_count, c.d_flags, ms.n_active);
    launch_markers(c, ms, q, theta, true);
    // the operator: fused stencil sweep, -S lambda, then -J v + K U and K^T lambda
    launch_apply_fluid<double>(c, x, y);
    if (c.nm == 0) {
        launch_zero_bodies<double>(c, y);
    } else {
        launch_spread<double>(c, ms, x, y, -1.0);
        launch_body_apply<double>(c, ms, nullptr, x, y);
    }
    HIP_OK(hipGetLastError());
    return RBFIB_OK;
}

}  // namespace rb

extern "C" int rbfib_apply_saddle_noalloc(const rbfib_grid *grid, const rbfib_bodies *bodies, const double *q,
                                          const double *theta, const double *x, double *y, void *hip_stream) {
    try {
        return rb::apply_noalloc(grid, bodies, q, theta, x, y, (hipStream_t)hip_stream);
    } catch (int code) {
        return code;
    } catch (...) {
        return RBFIB_EDEVICE;
    }
}

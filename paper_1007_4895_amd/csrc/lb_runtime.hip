// lb_runtime.hip -- host runtime behind include/lb.h.
//
// Owns no device memory: everything lives in the caller's workspace, carved
// up by ws_layout().  All work is enqueued on the caller's stream.  A time
// step is: one k_update launch per velocity set (work items = 64 columns x a
// strip of rows of that set; walls are handled there), then the projection
// of the halo-source nodes into the partner set (one thread per node and
// target population), then -- only where present -- row images and pressure
// columns, and in the interpolation/extrapolation interface mode the
// interface-row kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lb.h"
#include "lb_internal.hpp"
#include "lb_lists.hpp"
#include "lb_registry.hpp"
#include "lb_tables.hpp"

using namespace lbi;

namespace {

thread_local std::string g_err;

lb_status fail(lb_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return fail(LB_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

double xmax_of(int n) {
    switch (n) {
        case 3: return lbt::Tab<3>::xmax();
        case 4: return lbt::Tab<4>::xmax();
        case 6: return lbt::Tab<6>::xmax();
    }
    return 0.0;
}

void abscissae(int n, double *x, double *w) {
    auto cp = [&](const auto &r) {
        for (int p = 0; p < n; ++p) {
            x[p] = r.x[p];
            w[p] = r.w[p];
        }
    };
    if (n == 3) cp(lbt::Tab<3>::rule);
    if (n == 4) cp(lbt::Tab<4>::rule);
    if (n == 6) cp(lbt::Tab<6>::rule);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int esize_of(int storage) { return storage == LB_STORE_F64 ? 8 : storage == LB_STORE_F32 ? 4 : 2; }

struct Layout {
    int32_t pitch[2], rowbase[2];
    int64_t plane[2];
    size_t off_pop[2][2];   // [set][copy]
    size_t off_blo, off_bhi, off_oblo, off_obhi;
    size_t off_items[2], off_fin, off_proj, off_stage, off_mom, off_part, off_clw, off_clo;
    int maxitems, maxfin;
    size_t stage_elems;
    size_t total;
};

int ntiles_of(const lb_params &p) {
    int tw = p.tile_w > 0 ? p.tile_w : p.nx;
    return (p.nx + tw - 1) / tw;
}

Layout ws_layout(const lb_params &p) {
    Layout L{};
    const int eb = esize_of(p.storage);
    const int al = 128 / eb;
    const int nrow = p.ny + 1;
    const int n[2] = {p.n_low, p.n_high};
    size_t off = 0;
    // rows start on 128-byte lines, except for lattices narrower than a
    // line, whose rows are packed (16-byte steps) so that neighbouring rows
    // share lines and the footprint is not mostly padding
    const size_t row_al = size_t(p.nx + 4) * eb < 128 ? size_t(std::max(1, 16 / eb)) : size_t(al);
    for (int s = 0; s < 2; ++s) {
        L.pitch[s] = int32_t(align_up(size_t(p.nx) + 4, row_al));
        L.rowbase[s] = al;
        L.plane[s] = int64_t(align_up(size_t(al) + size_t(nrow + 4) * L.pitch[s], al));
        size_t bytes = size_t(n[s] * n[s]) * size_t(L.plane[s]) * eb;
        for (int c = 0; c < 2; ++c) {
            L.off_pop[s][c] = off;
            off = align_up(off + bytes, 256);
        }
    }
    const int nt = ntiles_of(p);
    const size_t nodes = size_t(nrow) * p.nx;
    L.off_blo = off; off = align_up(off + 4 * nt, 256);
    L.off_bhi = off; off = align_up(off + 4 * nt, 256);
    L.off_oblo = off; off = align_up(off + 4 * nt, 256);
    L.off_obhi = off; off = align_up(off + 4 * nt, 256);
    const int ngrp = (p.nx + 59) / 60;
    L.maxitems = 8 * (ngrp / 8 + 1) * (nrow + 4);
    for (int s = 0; s < 2; ++s) {
        L.off_items[s] = off;
        off = align_up(off + 16 * size_t(L.maxitems), 256);
    }
    L.maxfin = int(nodes);
    L.off_fin = off; off = align_up(off + 16 * nodes, 256);
    L.off_proj = off; off = align_up(off + 8 * nodes, 256);
    int qmax = std::max(std::max(n[0] * n[0], n[1] * n[1]), 3);
    L.stage_elems = size_t(qmax) * nodes;
    L.off_stage = off; off = align_up(off + 8 * L.stage_elems, 256);
    L.off_mom = off; off = align_up(off + 8 * 3 * nodes, 256);
    L.off_part = off; off = align_up(off + 8 * 3 * 1024, 256);
    L.off_clw = off; off = align_up(off + 2 * 5384, 256);
    L.off_clo = off; off = align_up(off + 4 * 6 * nodes, 256);
    L.total = off;
    return L;
}

const lbk::KernelSet *find_ks(int storage, int nS, int eqS, int nO, int eqO, int th = 0) {
    lbk::Registry r{};
    if (th) {
        if (storage == LB_STORE_F64) r = lbk::registry_f64_thermal();
        else if (storage == LB_STORE_F32) r = lbk::registry_f32_thermal();
        else return nullptr;
    } else {
        r = storage == LB_STORE_F64   ? lbk::registry_f64()
            : storage == LB_STORE_F32 ? lbk::registry_f32()
                                      : lbk::registry_bf16();
    }
    for (int k = 0; k < r.count; ++k) {
        const lbk::KernelSet &e = r.sets[k];
        if (e.nS == nS && e.eqS == eqS && e.nO == nO && e.eqO == eqO) return &e;
    }
    return nullptr;
}

const lbk::KernelSet *find_any(int nS, int eqS, int nO, int eqO) {
    for (int st = 0; st < 3; ++st)
        if (auto k = find_ks(st, nS, eqS, nO, eqO)) return k;
    return nullptr;
}

using lbl::host_reg;

// Hermite coefficients h_0..h_eq of the 1D Maxwellian factor at velocity u,
// temperature 1 + th: h_{k+1} = u h_k + k th h_{k-1} (u^k when th = 0)
void maxwell_coeffs(double u, double th, int eq, double *h) {
    h[0] = 1.0;
    for (int k = 1; k <= eq; ++k) h[k] = k >= 2 ? u * h[k - 1] + double(k - 1) * th * h[k - 2] : u;
}

// Diffuse-wall constants of a set (Sec. 3.2): S = f_eq(rho = 1, u_wall,
// T_wall) of the set's order (T_wall = 1 on isothermal lattices), stored as
// S' = S - w (computed without cancellation), K = sum_leaving |xi_y| w and
// D' = sum_leaving |xi_y| S', where the populations leaving the bottom wall
// have xi_y > 0 and those leaving the top wall xi_y < 0.
void wall_constants(int n, int eq, const double *x, const double *w, const double *uw, const double *Tw,
                    SetK &k) {
    for (int ws = 0; ws < 2; ++ws) {
        const double u = uw[2 * ws], v = uw[2 * ws + 1];
        double hu[8], hv[8];
        maxwell_coeffs(u, Tw[ws] - 1.0, eq, hu);
        maxwell_coeffs(v, Tw[ws] - 1.0, eq, hv);
        double K = 0.0, D = 0.0;
        for (int q = 0; q < n; ++q)
            for (int p = 0; p < n; ++p) {
                const int a = p + n * q;
                double s = 0.0;
                for (int kx = 0; kx <= eq; ++kx)
                    for (int m = 0; m + kx <= eq; ++m)
                        if (kx + m > 0)
                            s += hu[kx] * hv[m] * lbt::hermite(kx, x[p]) * lbt::hermite(m, x[q]) /
                                 (lbt::factorial(kx) * lbt::factorial(m));
                const double sp = w[p] * w[q] * s;
                k.sp[ws][a] = sp;
                k.spf[ws][a] = float(sp);
                const bool leaving = ws == 0 ? x[q] > 0.0 : x[q] < 0.0;
                if (leaving) {
                    K += std::fabs(x[q]) * w[p] * w[q];
                    D += std::fabs(x[q]) * sp;
                }
            }
        k.wK[ws] = K;
        k.wD[ws] = D;
        k.wKf[ws] = float(K);
        k.wDf[ws] = float(D);
    }
}

// ------------------------------------------------ generic (untemplated) kernels
// Sum over the 64 lanes of a wave by a fixed butterfly (xor 32, 16, ..., 1):
// every lane ends with the same, order-independent-of-scheduling total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sums of three per-node FP64 fields (rho, rho ux, rho uy): each thread
// accumulates a fixed strided subset, each wave reduces its lanes by a
// butterfly, and wave 0 adds the four wave totals in order; one partial
// per block.  The order never depends on timing, so the sums are
// deterministic.
__global__ __launch_bounds__(256) void k_sum3_partial(const double *a, const double *b, const double *c, int64_t n,
                                                      double *part) {
    __shared__ double sh[3][4];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        double r = a[k];
        s0 += r;
        s1 += r * b[k];
        s2 += r * c[k];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = s0;
        sh[1][w] = s1;
        sh[2][w] = s2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        part[q * 1024 + blockIdx.x] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
    }
}

// Final sums of the nb <= 1024 block partials, the same way (one block).
__global__ __launch_bounds__(256) void k_sum3_final(double *part, int nb) {
    __shared__ double sh[3][4];
    const int w = threadIdx.x >> 6;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) s += part[q * 1024 + b];
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) sh[q][w] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        part[q * 1024] = ((sh[q][0] + sh[q][1]) + sh[q][2]) + sh[q][3];
    }
}

// Per-tile bands from the indicator: bottom band = 1 + highest lower-half
// row with B > theta (mirrored at the top), clamped to [bmin, bmax].
__global__ void k_bands(const double *B, Geo g, double theta, int bmin, int bmax, int32_t *blo, int32_t *bhi) {
    __shared__ int slo, shi;
    const int t = blockIdx.x;
    if (threadIdx.x == 0) {
        slo = 0;
        shi = 0;
    }
    __syncthreads();
    const int half = g.ny / 2;
    const int c0 = t * g.tile_w, c1 = min(c0 + g.tile_w, g.nx);
    const int w = c1 - c0;
    int lo = 0, hi = 0;
    for (int k = threadIdx.x; k < w * (half + 1); k += blockDim.x) {
        int i = c0 + k % w, j = k / w;
        if (B[(int64_t)j * g.nx + i] > theta) lo = max(lo, j + 1);
        if (B[(int64_t)(g.ny - j) * g.nx + i] > theta) hi = max(hi, j + 1);
    }
    atomicMax(&slo, lo);
    atomicMax(&shi, hi);
    __syncthreads();
    if (threadIdx.x == 0) {
        blo[t] = min(max(slo, bmin), bmax);
        bhi[t] = min(max(shi, bmin), bmax);
    }
}

}  // namespace

struct lb_lattice {
    lb_params p;
    hipStream_t stream;
    char *ws;
    Layout lay;
    int n[2], eq[2], Q[2];
    Buf buf[2];
    SetK kconst[2];
    const lbk::KernelSet *ks[2];
    Geo geo;
    Phys ph;
    double dt, tau0, rho_shift, dshift;   // storage shift s0, ds (lbi::Shift)
    bool th;                              // thermal lattice
    double Tw[2];                         // wall temperatures (1 unless thermal)
    int ntiles, tile_w, cur;
    int64_t step;
    bool initialized;
    std::vector<int32_t> blo, bhi;
    int32_t *d_blo, *d_bhi, *d_oblo, *d_obhi;
    int32_t *d_items[2];
    int nitems[2];
    int32_t *d_fin;      // row images / pressure columns: (i, j, set, 0)
    int nfin;
    int32_t *d_proj;     // halo sources: (i, j), low-set nodes first
    int nproj[2];
    int strip[2];        // rows per work item per set (0 = automatic)
    int order[2];        // item order per set: 0 = XCD slabs row-major, 1 = column-major
    double *d_stage, *d_mom, *d_part;
    bool timing;
    int32_t timing_every = 1;   // in timing mode, events on every Nth step's update launches
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used;
    std::vector<int> ev_kind;   // per event pair: 1 = dominant update kernel, 0 = other update
    int64_t count[3];           // nodes per region: low, high, interface rows
    bool closure_on;            // learned closure in the lift
    bool closure_flags;         // the network's region flag in lb_update_regions
    uint16_t *d_clw;            // closure weights (bf16)
    float *d_clo;               // closure coefficients of the lifted nodes
    ClosureNorm cn;
    int dom;                    // set whose update moves the most bytes per step
    int64_t gen;                // bumped whenever the region map (work lists) changes
    bool merged;                // both sets' updates in one launch when the low set is D2Q9
    bool tuning;                // inside the autotuner (per-set kernels)
    bool concurrent;            // run the low set's kernels on a second stream
    hipStream_t side;           // that stream (created on first use)
    hipEvent_t efork, ejoin;
};

namespace {

NodeArgs node_args(const lb_lattice *L, int s, int copy) {
    NodeArgs a{};
    a.g = L->geo;
    a.ph = L->ph;
    a.self = L->buf[s];
    a.other = L->buf[1 - s];
    a.rho_shift = L->rho_shift;
    a.dshift = L->dshift;
    a.cur = copy;
    a.self_high = s;
    a.which = s;
    return a;
}

int node_grid(const lb_lattice *L) { return (L->geo.nrow * L->geo.nx + 255) / 256; }

// work items of set s: per 60-column group (the columns a block of the
// update kernel writes), the maximal runs of rows in which any column of
// the group belongs to the set, cut into strips; the list is ordered
// column-major so neighbouring strips are consecutive (and land on the same
// XCD through the kernel's mapping)
// maximal runs [j0, j1) of rows of set s per 60-column group (first column
// in runcol); returns the total number of rows
int set_runs(const lb_lattice *L, int s, std::vector<std::pair<int, int>> &runs, std::vector<int> &runcol) {
    const int nx = L->p.nx, ny = L->p.ny, nrow = ny + 1;
    const int want = s ? REG_HIGH : REG_LOW;
    const int ngrp = (nx + 59) / 60;
    int rows = 0;
    runs.clear();
    runcol.clear();
    std::vector<char> inset(nrow);
    for (int w = 0; w < ngrp; ++w) {
        const int i0 = 60 * w, i1 = std::min(i0 + 60, nx);
        const int t0 = L->ntiles == 1 ? 0 : i0 / L->tile_w, t1 = L->ntiles == 1 ? 0 : (i1 - 1) / L->tile_w;
        for (int j = 0; j < nrow; ++j) {
            inset[j] = 0;
            for (int t = t0; t <= t1; ++t)
                if (host_reg(L->blo[t], L->bhi[t], j, ny, L->p.iface) == want) inset[j] = 1;
        }
        int j = 0;
        while (j < nrow) {
            if (!inset[j]) {
                ++j;
                continue;
            }
            int j1 = j;
            while (j1 < nrow && inset[j1]) ++j1;
            runs.push_back({j, j1});
            runcol.push_back(i0);
            rows += j1 - j;
            j = j1;
        }
    }
    return rows;
}

// rows per item when none is set: enough blocks to give every CU a few
// resident ones
int auto_strip(int64_t rows) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return int(std::max<int64_t>(1, std::min<int64_t>(16, rows / (8 * cus))));
}

int build_items(const lb_lattice *L, int s, std::vector<int32_t> &out) {
    out.clear();
    const int ngrp = (L->p.nx + 59) / 60;
    std::vector<std::pair<int, int>> runs;
    std::vector<int> runcol;
    const int rows = set_runs(L, s, runs, runcol);
    int strip = L->strip[s];
    if (strip <= 0) strip = auto_strip(rows);
    // Item order: the kernel gives XCD x the items [x * chunk, (x + 1) * chunk).
    // Each XCD gets a contiguous slab of column groups, and inside the slab
    // the strips are ordered row-major: blocks running together touch
    // neighbouring groups of the same rows (they share the edge cache lines
    // of their overlapping loads in that XCD's L2, and HBM sees long runs),
    // and the next strip up finds its two halo rows still in the same L2.
    // Slabs are padded with empty items to a common length.
    struct It { int slab, j0, i0, j1; };
    std::vector<It> v;
    for (size_t r = 0; r < runs.size(); ++r)
        for (int j = runs[r].first; j < runs[r].second; j += strip) {
            const int g = runcol[r] / 60;
            v.push_back({int(int64_t(g) * 8 / ngrp), j, runcol[r], std::min(j + strip, runs[r].second)});
        }
    if (ngrp < 8 || L->order[s] == 1) {
        // too few column groups for one per XCD (or column-major order
        // requested): cut the ordered list into 8 contiguous pieces instead
        const bool cm = L->order[s] == 1;
        std::sort(v.begin(), v.end(), [cm](const It &a, const It &b) {
            if (cm) return a.i0 != b.i0 ? a.i0 < b.i0 : a.j0 < b.j0;
            return a.j0 != b.j0 ? a.j0 < b.j0 : a.i0 < b.i0;
        });
        for (size_t k = 0; k < v.size(); ++k) v[k].slab = int(k * 8 / v.size());
    }
    const bool colmajor = L->order[s] == 1;
    std::sort(v.begin(), v.end(), [colmajor](const It &a, const It &b) {
        if (a.slab != b.slab) return a.slab < b.slab;
        if (colmajor) return a.i0 != b.i0 ? a.i0 < b.i0 : a.j0 < b.j0;
        if (a.j0 != b.j0) return a.j0 < b.j0;
        return a.i0 < b.i0;
    });
    int per[8] = {0};
    for (auto &e : v) per[e.slab]++;
    int chunk = 0;
    for (int x = 0; x < 8; ++x) chunk = std::max(chunk, per[x]);
    out.assign(size_t(8) * chunk * 4, 0);
    int fill[8] = {0};
    for (auto &e : v) {
        int k = e.slab * chunk + fill[e.slab]++;
        out[4 * k] = e.i0;
        out[4 * k + 1] = e.j0;
        out[4 * k + 2] = e.j1;
        out[4 * k + 3] = 0;
    }
    return int(out.size() / 4);
}


// Per-step lists of a lattice (lbl::build_lists on its decomposition).
int build_lists(const lb_lattice *L, std::vector<int32_t> &fin, std::vector<int32_t> &proj, int nproj[2]) {
    const lbl::Decomp D{L->p.nx, L->p.ny, L->p.xbc, L->p.ybc, L->p.iface, L->ntiles, L->tile_w,
                        L->blo.data(), L->bhi.data()};
    return lbl::build_lists(D, fin, proj, nproj);
}

lb_status upload_regions(lb_lattice *L) {
    HIPCHK(hipMemcpyAsync(L->d_blo, L->blo.data(), 4 * L->ntiles, hipMemcpyHostToDevice, L->stream));
    HIPCHK(hipMemcpyAsync(L->d_bhi, L->bhi.data(), 4 * L->ntiles, hipMemcpyHostToDevice, L->stream));
    std::vector<int32_t> v;
    for (int s = 0; s < 2; ++s) {
        L->nitems[s] = build_items(L, s, v);
        if (L->nitems[s] > L->lay.maxitems) return fail(LB_EINVAL, "too many work items");
        if (L->nitems[s])
            HIPCHK(hipMemcpyAsync(L->d_items[s], v.data(), v.size() * 4, hipMemcpyHostToDevice, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    for (int k = 0; k < 3; ++k) L->count[k] = 0;
    for (int j = 0; j <= L->p.ny; ++j)
        for (int t = 0; t < L->ntiles; ++t) {
            int w = std::min(L->tile_w, L->p.nx - t * L->tile_w);
            L->count[host_reg(L->blo[t], L->bhi[t], j, L->p.ny, L->p.iface)] += w;
        }
    L->dom = double(L->Q[1]) * L->count[1] > double(L->Q[0]) * L->count[0] ? 1 : 0;
    std::vector<int32_t> pv;
    L->nfin = build_lists(L, v, pv, L->nproj);
    if (L->nfin) HIPCHK(hipMemcpyAsync(L->d_fin, v.data(), v.size() * 4, hipMemcpyHostToDevice, L->stream));
    if (!pv.empty()) HIPCHK(hipMemcpyAsync(L->d_proj, pv.data(), pv.size() * 4, hipMemcpyHostToDevice, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    L->gen++;
    return LB_OK;
}

lb_status check_bands(const lb_lattice *L, const int32_t *lo, const int32_t *hi) {
    for (int t = 0; t < L->ntiles; ++t) {
        if (lo[t] < 0 || hi[t] < 0 || lo[t] > L->p.ny + 1 || hi[t] > L->p.ny + 1)
            return fail(LB_EINVAL, "band out of range in tile %d", t);
        if (L->p.iface == LB_IFACE_PAPER) {
            if (lo[t] != lo[0] || hi[t] != hi[0])
                return fail(LB_EINVAL, "the interpolation interface needs the same bands in every tile");
            if (lo[t] + hi[t] + 3 > L->p.ny + 1 && (lo[t] > 0 || hi[t] > 0))
                return fail(LB_EINVAL, "bands leave no low-order rows between the interface rows");
        }
    }
    return LB_OK;
}

void set_geo(lb_lattice *L) {
    L->geo.nx = L->p.nx;
    L->geo.ny = L->p.ny;
    L->geo.nrow = L->p.ny + 1;
    L->geo.tile_w = L->tile_w;
    L->geo.ntiles = L->ntiles;
    L->geo.xbc = L->p.xbc;
    L->geo.ybc = L->p.ybc;
    L->geo.iface = L->p.iface;
    L->geo.blo = L->d_blo;
    L->geo.bhi = L->d_bhi;
}

lb_status refresh_all(lb_lattice *L, int recompute_iface) {
    const int grid = node_grid(L);
    for (int s = 0; s < 2; ++s) L->ks[s]->refresh(node_args(L, s, L->cur), grid, L->stream);
    if (L->p.iface == LB_IFACE_PAPER)
        L->ks[0]->paper_iface(node_args(L, 0, L->cur), L->cur, recompute_iface, (2 * L->p.nx + 255) / 256,
                              L->stream);
    HIPCHK(hipGetLastError());
    return LB_OK;
}

hipEvent_t next_event(lb_lattice *L) {
    if (L->ev_used == L->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        L->ev_pool.push_back(e);
    }
    return L->ev_pool[L->ev_used++];
}

// seed of the stochastic rounding of step n (bf16 storage); the kernels hash
// it with the row and the population
uint32_t step_seed(int64_t n) { return uint32_t(uint64_t(n) * 0x9e3779b97f4a7c15ull >> 32); }

// The two sets are independent within a step until the interface: the low
// set's update and its projection into the high set's halo run on a second
// stream, concurrently with the high set's update and its projection into
// the low set's halo (disjoint rows of disjoint buffers); the streams join
// before the finish pass.
lb_status make_side_stream(lb_lattice *L) {
    HIPCHK(hipStreamCreateWithFlags(&L->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&L->efork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&L->ejoin, hipEventDisableTiming));
    return LB_OK;
}

// Wall constants of both sets for the wall velocities of time level
// t = (step + 1) dt: the oscillating bottom wall (oscillatory Couette flow,
// Sec. 3.5) adds u_osc sin(omega_osc t) to its x velocity.
void set_wall_constants(lb_lattice *L, int64_t step) {
    double uw[4];
    for (int k = 0; k < 4; ++k) uw[k] = L->p.u_wall[k];
    if (L->p.u_osc != 0.0) uw[0] += L->p.u_osc * std::sin(L->p.omega_osc * double(step + 1) * L->dt);
    for (int s = 0; s < 2; ++s) {
        double x[8] = {0}, w[8] = {0};
        abscissae(L->n[s], x, w);
        wall_constants(L->n[s], L->eq[s], x, w, uw, L->Tw, L->kconst[s]);
    }
}

// Thermal lattices whose low set is D2Q9 never launch that set's update on
// its own (k_update): a test of separate launches on such a lattice hung
// once on the GPU and the cause has not been found, so that kernel stays
// unused.  Their D2Q9 items always run in the merged kernel's D2Q9 branch
// (the same device code), and the calls that would need the separate
// launch (merged update off, concurrent streams, the per-set timings of
// the autotuner) are refused.
bool d2q9_alone_off(const lb_lattice *L) { return L->th && L->n[0] == 3; }

lb_status one_step(lb_lattice *L) {
    if (L->p.u_osc != 0.0) set_wall_constants(L, L->step);
    StepArgs a{};
    a.g = L->geo;
    a.ph = L->ph;
    a.rho_shift = L->rho_shift;
    a.dshift = L->dshift;
    a.cur = L->cur;
    a.seed = step_seed(L->step);
    const bool par = L->concurrent && !L->timing && L->nitems[0] && L->nitems[1] && L->p.iface == LB_IFACE_HERMITE;
    // (timing mode records events around the update launches of every Nth
    // step; the launches themselves are the same in every step)
    const bool timed_now = L->timing && L->step % L->timing_every == 0;
    if (par && !L->side) {
        lb_status st = make_side_stream(L);
        if (st != LB_OK) return st;
    }
    hipStream_t sl = par ? L->side : L->stream;   // stream of the low set's kernels
    if (par) {
        HIPCHK(hipEventRecord(L->efork, L->stream));
        HIPCHK(hipStreamWaitEvent(L->side, L->efork, 0));
    }
    // (thermal lattices with a D2Q9 low set always take the merged launch,
    // with no high-set blocks when that set is empty: their D2Q9 update runs
    // only in the merged kernel's D2Q9 branch -- see d2q9_alone_off)
    const bool merge = L->ks[0]->update_pair && L->nitems[0] &&
                       (d2q9_alone_off(L) || (L->merged && !par && !L->tuning && L->nitems[1]));
    if (merge) {
        StepArgs sa[2] = {a, a};
        for (int s = 0; s < 2; ++s) {
            sa[s].self = L->buf[s];
            sa[s].other = L->buf[1 - s];
            sa[s].ks = L->kconst[s];
            sa[s].self_high = s;
            sa[s].items = L->d_items[s];
            sa[s].nitems = L->nitems[s];
            sa[s].chunk = (L->nitems[s] + 7) / 8;
        }
        const int sp = L->ks[0]->pair_split;
        const int nb_h = L->nitems[1] ? 8 * sa[1].chunk : 0, nb_l = 8 * ((sa[0].chunk + sp - 1) / sp);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed_now) {
            e0 = next_event(L);
            e1 = next_event(L);
            if (!e0 || !e1) return fail(LB_EDEVICE, "event creation failed");
            L->ev_kind.push_back(L->dom);   // the only update launch of the step
        }
        L->ks[0]->update_pair(sa[0], sa[1], nb_h, nb_l, L->stream, e0, e1);
    }
    for (int s = 0; s < 2 && !merge; ++s) {
        if (!L->nitems[s]) continue;
        a.self = L->buf[s];
        a.other = L->buf[1 - s];
        a.ks = L->kconst[s];
        a.self_high = s;
        a.items = L->d_items[s];
        a.nitems = L->nitems[s];
        a.chunk = (a.nitems + 7) / 8;
        if (timed_now) {
            hipEvent_t e0 = next_event(L), e1 = next_event(L);
            if (!e0 || !e1) return fail(LB_EDEVICE, "event creation failed");
            L->ev_kind.push_back(s);
            L->ks[s]->update_timed(a, 8 * a.chunk, L->stream, e0, e1);
        } else {
            L->ks[s]->update(a, 8 * a.chunk, s ? L->stream : sl);
        }
    }
    a.self = L->buf[0];
    a.other = L->buf[1];
    bool fin_done = false;
    if (L->nproj[0] + L->nproj[1]) {
        a.items = L->d_proj;
        a.nitems = L->nproj[0];
        a.chunk = L->nproj[1];
        a.clo = nullptr;
        // a learned-closure step runs the inference inside the projection
        // launch (one launch fewer per step); the two-stream mode keeps the
        // inference launch before the projection into the high set
        const bool fused = L->closure_on && L->nproj[0] && !par && L->ks[0]->project_closure;
        if (L->closure_on && L->nproj[0]) {
            a.clw = L->d_clw;
            a.cn = L->cn;
            if (!fused) {
                a.clo = L->d_clo;
                L->ks[0]->closure_infer(a, (L->nproj[0] + lbi::CLOSURE_NB - 1) / lbi::CLOSURE_NB, sl);
            }
        }
        if (fused) {
            const int nbl = (L->nproj[0] + lbi::CLOSURE_NB - 1) / lbi::CLOSURE_NB;
            const int nbd = int((int64_t(L->nproj[1]) * L->n[0] + 63) / 64);
            const int qm = std::max(L->Q[0], L->Q[1]);
            const int nbf = int((int64_t(L->nfin) * qm + 63) / 64);
            L->ks[0]->project_closure(a, L->d_fin, L->nfin, nbl, nbd, nbl + nbd + nbf, L->stream);
            fin_done = true;
        } else if (par) {
            // low -> high on the low set's stream, high -> low on the other
            StepArgs up = a, down = a;
            up.chunk = 0;
            down.items = L->d_proj + 2 * L->nproj[0];
            down.nitems = 0;
            down.clo = nullptr;
            if (L->nproj[0]) L->ks[0]->project_halo(up, int((int64_t(L->nproj[0]) * L->n[1] + 127) / 128), sl);
            if (L->nproj[1])
                L->ks[0]->project_halo(down, int((int64_t(L->nproj[1]) * L->n[0] + 127) / 128), L->stream);
        } else {
            // one thread per (node, target column); with a finish list, its
            // pass joins the same launch (one thread per node and population)
            const int64_t nt = int64_t(L->nproj[0]) * L->n[1] + int64_t(L->nproj[1]) * L->n[0];
            const int nbp = int((nt + 127) / 128);
            if (L->nfin) {
                const int qm = std::max(L->Q[0], L->Q[1]);
                const int nbf = int((int64_t(L->nfin) * qm + 127) / 128);
                L->ks[0]->project_finish(a, L->d_fin, L->nfin, nbp, nbp + nbf, L->stream);
                fin_done = true;
            } else {
                L->ks[0]->project_halo(a, nbp, L->stream);
            }
        }
    }
    if (par) {
        HIPCHK(hipEventRecord(L->ejoin, L->side));
        HIPCHK(hipStreamWaitEvent(L->stream, L->ejoin, 0));
    }
    if (L->nfin && !fin_done) {
        a.items = L->d_fin;
        a.nitems = L->nfin;
        const int qm = std::max(L->Q[0], L->Q[1]);   // one thread per (node, population)
        L->ks[0]->finish(a, int((int64_t(L->nfin) * qm + 127) / 128), L->stream);
    }
    if (L->p.iface == LB_IFACE_PAPER)
        L->ks[0]->paper_iface(node_args(L, 0, L->cur ^ 1), L->cur ^ 1, 1, (2 * L->p.nx + 255) / 256, L->stream);
    L->cur ^= 1;
    L->step++;
    return LB_OK;
}

}  // namespace

lb_status lb_internal_fail(lb_status s, const char *msg) { return fail(s, "%s", msg); }

extern "C" {

const char *lb_last_error(void) { return g_err.c_str(); }

lb_status lb_params_default(lb_params *p) {
    if (!p) return fail(LB_EINVAL, "null params");
    memset(p, 0, sizeof(*p));
    p->nx = 64;
    p->ny = 64;
    p->n_low = p->n_high = 3;
    p->eq_low = p->eq_high = 2;
    p->tau_mode = LB_TAU_CONST;
    p->xbc = LB_XBC_PERIODIC;
    p->ybc = LB_YBC_WALLS;
    p->iface = LB_IFACE_HERMITE;
    p->storage = LB_STORE_F64;
    p->kn = 0.1;
    p->rho_ref = 1.0;
    p->cfl = 0.5;
    p->rho_in = p->rho_out = 1.0;
    p->T_wall[0] = p->T_wall[1] = 1.0;
    return LB_OK;
}

static lb_status validate(const lb_params *p) {
    if (!p) return fail(LB_EINVAL, "null params");
    if (p->nx < 2 || p->ny < 4) return fail(LB_EINVAL, "lattice too small (nx >= 2, ny >= 4)");
    if (size_t(p->nx) * size_t(p->ny + 1) > (size_t(1) << 31)) return fail(LB_EINVAL, "lattice too large");
    const int n[2] = {p->n_low, p->n_high}, eq[2] = {p->eq_low, p->eq_high};
    const int fo[2] = {p->force_low, p->force_high};
    for (int s = 0; s < 2; ++s) {
        if (n[s] != 3 && n[s] != 4 && n[s] != 6)
            return fail(LB_EUNSUPPORTED, "velocity set with %d points per axis not built (3, 4, 6)", n[s]);
        // quadrature of degree 2n-1 resolves the equilibrium up to order n-1
        if (eq[s] < 1 || eq[s] > n[s] - 1)
            return fail(LB_EINVAL, "equilibrium order %d outside [1, %d] for D2Q%d", eq[s], n[s] - 1, n[s] * n[s]);
        if (fo[s] != 0 && fo[s] != eq[s])
            return fail(LB_EUNSUPPORTED, "force order must equal the equilibrium order");
    }
    if (p->storage < 0 || p->storage > 2) return fail(LB_EINVAL, "bad storage");
    if (p->iface != LB_IFACE_HERMITE && p->iface != LB_IFACE_PAPER) return fail(LB_EINVAL, "bad interface");
    if (p->xbc != LB_XBC_PERIODIC && p->xbc != LB_XBC_PRESSURE) return fail(LB_EINVAL, "bad xbc");
    if (p->ybc != LB_YBC_WALLS && p->ybc != LB_YBC_PERIODIC && p->ybc != LB_YBC_SHEAR)
        return fail(LB_EINVAL, "bad ybc");
    if (!std::isfinite(p->shear_top)) return fail(LB_EINVAL, "shear rate must be finite");
    if (p->tau_mode != LB_TAU_CONST && p->tau_mode != LB_TAU_RHO) return fail(LB_EINVAL, "bad tau mode");
    if (!(p->kn > 0) || !(p->rho_ref > 0)) return fail(LB_EINVAL, "kn and rho_ref must be positive");
    if (!std::isfinite(p->u_osc) || !std::isfinite(p->omega_osc))
        return fail(LB_EINVAL, "oscillating wall amplitude and frequency must be finite");
    if (p->u_osc != 0.0 && p->ybc == LB_YBC_PERIODIC) return fail(LB_EINVAL, "an oscillating wall needs walls");
    const int tw = p->tile_w > 0 ? p->tile_w : p->nx;
    if (tw != p->nx && tw % 64 != 0) return fail(LB_EINVAL, "tile_w must be a multiple of 64 (or nx)");
    if (p->xbc == LB_XBC_PRESSURE && p->nx < 4) return fail(LB_EINVAL, "pressure boundary needs nx >= 4");
    const double xm = std::max(xmax_of(n[0]), xmax_of(n[1]));
    double dt = p->dt > 0 ? p->dt : p->cfl * (1.0 / xm);
    if (p->dt <= 0 && !(p->cfl > 0 && p->cfl <= 0.5)) return fail(LB_EINVAL, "cfl must be in (0, 0.5]");
    if (dt * xm > 1.0 + 1e-12) return fail(LB_EINVAL, "Courant number above 1");
    const double tau0 = p->kn * p->ny;
    if (dt > tau0) return fail(LB_EINVAL, "time step %g above the relaxation time %g", dt, tau0);
    Layout L = ws_layout(*p);
    for (int s = 0; s < 2; ++s)
        if (int64_t(n[s] * n[s]) * L.plane[s] * esize_of(p->storage) >= (int64_t(1) << 31))
            return fail(LB_EINVAL, "one set's populations exceed 2 GiB per copy");
    if (p->thermal != 0 && p->thermal != 1) return fail(LB_EINVAL, "thermal is 0 or 1");
    if (p->thermal) {
        for (int k = 0; k < 2; ++k)
            if (!(p->T_wall[k] > 0.0) || !std::isfinite(p->T_wall[k]))
                return fail(LB_EINVAL, "wall temperatures must be positive and finite");
        if (p->storage == LB_STORE_BF16) return fail(LB_EUNSUPPORTED, "thermal lattices are built for FP64 and FP32");
    }
    const int st = p->storage, th = p->thermal;
    if (!find_ks(st, n[0], eq[0], n[1], eq[1], th) || !find_ks(st, n[1], eq[1], n[0], eq[0], th))
        return fail(LB_EUNSUPPORTED, "no %skernels built for D2Q%d(order %d)/D2Q%d(order %d) with storage %d",
                    th ? "thermal " : "", n[0] * n[0], eq[0], n[1] * n[1], eq[1], st);
    return LB_OK;
}

size_t lb_workspace_bytes(const lb_params *p) {
    if (validate(p) != LB_OK) return 0;
    return ws_layout(*p).total;
}

lb_status lb_create_lattice(const lb_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                            lb_lattice **out) {
    if (!out) return fail(LB_EINVAL, "null output handle");
    *out = nullptr;
    lb_status st = validate(p);
    if (st != LB_OK) return st;
    Layout lay = ws_layout(*p);
    if (!dev_workspace || bytes < lay.total)
        return fail(LB_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, lay.total);
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return fail(LB_EINVAL, "workspace not 256-byte aligned");
    lb_lattice *L = new lb_lattice();
    L->p = *p;
    L->stream = reinterpret_cast<hipStream_t>(hip_stream);
    L->concurrent = false;
    L->merged = true;
    L->tuning = false;
    L->side = nullptr;
    L->efork = L->ejoin = nullptr;
    L->ws = reinterpret_cast<char *>(dev_workspace);
    L->lay = lay;
    L->n[0] = p->n_low;
    L->n[1] = p->n_high;
    L->eq[0] = p->eq_low;
    L->eq[1] = p->eq_high;
    for (int s = 0; s < 2; ++s) {
        L->Q[s] = L->n[s] * L->n[s];
        for (int c = 0; c < 2; ++c) L->buf[s].base[c] = L->ws + lay.off_pop[s][c];
        L->buf[s].plane = lay.plane[s];
        L->buf[s].pitch = lay.pitch[s];
        L->buf[s].rowbase = lay.rowbase[s];
    }
    L->th = p->thermal != 0;
    L->Tw[0] = L->th ? p->T_wall[0] : 1.0;
    L->Tw[1] = L->th ? p->T_wall[1] : 1.0;
    L->ks[0] = find_ks(p->storage, L->n[0], L->eq[0], L->n[1], L->eq[1], L->th);
    L->ks[1] = find_ks(p->storage, L->n[1], L->eq[1], L->n[0], L->eq[0], L->th);
    const double xm = std::max(xmax_of(L->n[0]), xmax_of(L->n[1]));
    L->dt = p->dt > 0 ? p->dt : p->cfl * (1.0 / xm);
    L->tau0 = p->kn * p->ny;
    // storage reference (lbi::Shift): 0 for FP64; rho_ref for FP32 / BF16,
    // or, for a pressure-driven lattice, the imposed linear density ramp at
    // the centre of each group of SHIFT_GROUP columns, so that the stored
    // deviations carry no density ramp
    L->rho_shift = p->storage == LB_STORE_F64 ? 0.0 : p->rho_ref;
    L->dshift = 0.0;
    if (p->storage != LB_STORE_F64 && p->xbc == LB_XBC_PRESSURE && p->rho_in != p->rho_out) {
        const double slope = (p->rho_out - p->rho_in) / double(p->nx - 1);
        L->rho_shift = p->rho_in + slope * 0.5 * double(lbi::SHIFT_GROUP - 1);
        L->dshift = slope * double(lbi::SHIFT_GROUP);
    }
    L->tile_w = p->tile_w > 0 ? p->tile_w : p->nx;
    L->ntiles = ntiles_of(*p);
    for (int s = 0; s < 2; ++s) {
        double x[8] = {0}, w[8] = {0};
        abscissae(L->n[s], x, w);
        wall_constants(L->n[s], L->eq[s], x, w, p->u_wall, L->Tw, L->kconst[s]);
        for (int q = 0; q < 8; ++q) {
            double nu = x[q] * L->dt, an = std::fabs(nu);
            L->kconst[s].nu[q] = nu;
            L->kconst[s].kk[q] = 0.5 * an * (1.0 - an);
            L->kconst[s].nuf[q] = float(nu);
            L->kconst[s].kkf[q] = float(0.5 * an * (1.0 - an));
        }
    }
    L->ph = Phys{};
    L->ph.dt = L->dt;
    L->ph.omega0 = L->dt / L->tau0;
    L->ph.rho_ref = p->rho_ref;
    L->ph.rho_in = p->rho_in;
    L->ph.rho_out = p->rho_out;
    L->ph.gx = p->gx;
    L->ph.gy = p->gy;
    for (int k = 0; k < 4; ++k) L->ph.uw[k] = p->u_wall[k];
    L->ph.shear = p->ybc == LB_YBC_SHEAR ? p->shear_top : 0.0;
    L->ph.tau_mode = p->tau_mode;
    L->ph.kn = p->kn;
    L->d_blo = reinterpret_cast<int32_t *>(L->ws + lay.off_blo);
    L->d_bhi = reinterpret_cast<int32_t *>(L->ws + lay.off_bhi);
    L->d_oblo = reinterpret_cast<int32_t *>(L->ws + lay.off_oblo);
    L->d_obhi = reinterpret_cast<int32_t *>(L->ws + lay.off_obhi);
    for (int s = 0; s < 2; ++s) L->d_items[s] = reinterpret_cast<int32_t *>(L->ws + lay.off_items[s]);
    L->d_fin = reinterpret_cast<int32_t *>(L->ws + lay.off_fin);
    L->d_proj = reinterpret_cast<int32_t *>(L->ws + lay.off_proj);
    L->d_stage = reinterpret_cast<double *>(L->ws + lay.off_stage);
    L->d_mom = reinterpret_cast<double *>(L->ws + lay.off_mom);
    L->d_part = reinterpret_cast<double *>(L->ws + lay.off_part);
    L->d_clw = reinterpret_cast<uint16_t *>(L->ws + lay.off_clw);
    L->d_clo = reinterpret_cast<float *>(L->ws + lay.off_clo);
    L->strip[0] = L->strip[1] = 0;
    L->order[0] = L->order[1] = 0;
    L->cur = 0;
    L->step = 0;
    L->blo.assign(L->ntiles, 0);
    L->bhi.assign(L->ntiles, 0);
    set_geo(L);
    st = upload_regions(L);
    if (st != LB_OK) {
        delete L;
        return st;
    }
    *out = L;
    return LB_OK;
}

void lb_destroy_lattice(lb_lattice *L) {
    if (!L) return;
    if (L->side) {
        (void)hipStreamSynchronize(L->side);
        (void)hipStreamDestroy(L->side);
        (void)hipEventDestroy(L->efork);
        (void)hipEventDestroy(L->ejoin);
    }
    for (auto e : L->ev_pool) (void)hipEventDestroy(e);
    delete L;
}

lb_status lb_get_info(const lb_lattice *L, double *dt, double *tau0, int32_t *ntiles) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (dt) *dt = L->dt;
    if (tau0) *tau0 = L->tau0;
    if (ntiles) *ntiles = L->ntiles;
    return LB_OK;
}

lb_status lb_set_regions(lb_lattice *L, const int32_t *lo, const int32_t *hi) {
    if (!L || !lo || !hi) return fail(LB_EINVAL, "null argument");
    lb_status st = check_bands(L, lo, hi);
    if (st != LB_OK) return st;
    L->blo.assign(lo, lo + L->ntiles);
    L->bhi.assign(hi, hi + L->ntiles);
    st = upload_regions(L);
    if (st != LB_OK) return st;
    if (L->initialized) return refresh_all(L, 1);
    return LB_OK;
}

lb_status lb_get_regions(const lb_lattice *L, int32_t *lo, int32_t *hi) {
    if (!L || !lo || !hi) return fail(LB_EINVAL, "null argument");
    std::copy(L->blo.begin(), L->blo.end(), lo);
    std::copy(L->bhi.begin(), L->bhi.end(), hi);
    return LB_OK;
}

lb_status lb_region_counts(const lb_lattice *L, int64_t counts[3]) {
    if (!L || !counts) return fail(LB_EINVAL, "null argument");
    for (int k = 0; k < 3; ++k) counts[k] = L->count[k];
    return LB_OK;
}

lb_status lb_set_strip_rows(lb_lattice *L, int32_t rows) {
    if (!L || rows < 0 || rows > 1024) return fail(LB_EINVAL, "strip rows in [0, 1024] (0 = automatic)");
    L->strip[0] = L->strip[1] = rows;
    return upload_regions(L);
}

lb_status lb_set_work_shape(lb_lattice *L, const int32_t rows[2], const int32_t order[2]) {
    if (!L || !rows || !order) return fail(LB_EINVAL, "null argument");
    for (int s = 0; s < 2; ++s) {
        if (rows[s] < 0 || rows[s] > 1024) return fail(LB_EINVAL, "strip rows in [0, 1024] (0 = automatic)");
        if (order[s] != 0 && order[s] != 1) return fail(LB_EINVAL, "item order is 0 or 1");
    }
    for (int s = 0; s < 2; ++s) {
        L->strip[s] = rows[s];
        L->order[s] = order[s];
    }
    return upload_regions(L);
}

lb_status lb_get_work_shape(const lb_lattice *L, int32_t rows[2], int32_t order[2]) {
    if (!L || !rows || !order) return fail(LB_EINVAL, "null argument");
    for (int s = 0; s < 2; ++s) {
        rows[s] = L->strip[s];
        order[s] = L->order[s];
    }
    return LB_OK;
}

lb_status lb_get_strip_rows(const lb_lattice *L, int32_t rows[2]) {
    if (!L || !rows) return fail(LB_EINVAL, "null argument");
    rows[0] = L->strip[0];
    rows[1] = L->strip[1];
    return LB_OK;
}

lb_status lb_autotune(lb_lattice *L, int32_t steps, int32_t rows_out[2]) {
    if (!L || steps < 1) return fail(LB_EINVAL, "bad argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    if (d2q9_alone_off(L))
        return fail(LB_EUNSUPPORTED, "no autotuner for thermal lattices with a D2Q9 low set (per-set timings)");
    // the trials advance the lattice: keep the state and restore it after
    std::vector<char> saved(lb_state_bytes(L));
    lb_status st = lb_get_state(L, saved.data(), saved.size());
    if (st != LB_OK) return st;
    const int cur0 = L->cur;
    L->tuning = true;   // time each set's kernel on its own
    static const int cand[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    for (int s = 0; s < 2; ++s) {
        if (!L->count[s]) continue;
        double best = 1e300;
        int best_rows = 1, best_order = 0;
        for (int cc = 0; cc < 2 * int(sizeof(cand) / sizeof(cand[0])); ++cc) {
            const int c = cand[cc >> 1], ord = cc & 1;
            L->strip[s] = c;
            L->order[s] = ord;
            if ((st = upload_regions(L)) != LB_OK) return st;
            // timed twice, the faster pass counting
            double t = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                L->timing = true;
                L->timing_every = 1;
                L->ev_used = 0;
                L->ev_kind.clear();
                for (int k = 0; k < steps; ++k)
                    if ((st = one_step(L)) != LB_OK) return st;
                HIPCHK(hipStreamSynchronize(L->stream));
                double tr = 0;
                for (size_t k = 0; k < L->ev_kind.size(); ++k) {
                    if (L->ev_kind[k] != s) continue;
                    float ms = 0;
                    HIPCHK(hipEventElapsedTime(&ms, L->ev_pool[2 * k], L->ev_pool[2 * k + 1]));
                    tr += ms;
                }
                t = std::min(t, tr);
            }
            if (t < best) {
                best = t;
                best_rows = c;
                best_order = ord;
            }
        }
        L->strip[s] = best_rows;
        L->order[s] = best_order;
    }
    L->timing = false;
    L->tuning = false;
    L->ev_used = 0;
    L->ev_kind.clear();
    // then the whole step as it runs (both sets' updates merged or in turn,
    // the projection): strips next to the per-set choices, each timed twice
    // over `steps` steps, the faster time counting
    if (L->count[0] && L->count[1]) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const int p0 = L->strip[0], p1 = L->strip[1];
        double best = 1e300;
        int b0 = p0, b1 = p1;
        for (int a = std::max(1, p0 - 1); a <= p0 + 1 && st == LB_OK; ++a)
            for (int b = std::max(1, p1 - 1); b <= p1 + 1 && st == LB_OK; ++b) {
                L->strip[0] = a;
                L->strip[1] = b;
                if ((st = upload_regions(L)) != LB_OK) break;
                for (int rep = 0; rep < 2 && st == LB_OK; ++rep) {
                    if (hipEventRecord(e0, L->stream) != hipSuccess) st = fail(LB_EDEVICE, "event record failed");
                    for (int k = 0; k < steps && st == LB_OK; ++k) st = one_step(L);
                    if (st != LB_OK) break;
                    float ms = 0;
                    if (hipEventRecord(e1, L->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                        st = fail(LB_EDEVICE, "event timing failed");
                    else if (ms < best) {
                        best = ms;
                        b0 = a;
                        b1 = b;
                    }
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != LB_OK) return st;
        L->strip[0] = b0;
        L->strip[1] = b1;
    }
    if ((st = upload_regions(L)) != LB_OK) return st;
    L->cur = cur0;
    st = lb_set_state(L, saved.data(), saved.size());
    if (rows_out) {
        rows_out[0] = L->strip[0];
        rows_out[1] = L->strip[1];
    }
    return st;
}

lb_status lb_init_equilibrium_thermal(lb_lattice *L, const double *rho, const double *ux, const double *uy,
                                      const double *T) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (T && !L->th) return fail(LB_EINVAL, "a temperature field needs a thermal lattice");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    const int nf = T ? 4 : 3;   // the staging area holds at least 9 fields
    std::vector<double> h(nf * N);
    for (size_t k = 0; k < N; ++k) {
        h[k] = rho ? rho[k] : L->p.rho_ref;
        h[N + k] = ux ? ux[k] : 0.0;
        h[2 * N + k] = uy ? uy[k] : 0.0;
        if (T) h[3 * N + k] = T[k];
    }
    HIPCHK(hipMemcpyAsync(L->d_stage, h.data(), 8 * nf * N, hipMemcpyHostToDevice, L->stream));
    const int grid = node_grid(L);
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.in0 = L->d_stage;
        a.in1 = L->d_stage + N;
        a.in2 = L->d_stage + 2 * N;
        a.in3 = T ? L->d_stage + 3 * N : nullptr;
        L->ks[s]->init_eq(a, grid, L->stream);
    }
    lb_status st = refresh_all(L, 1);
    if (st != LB_OK) return st;
    HIPCHK(hipStreamSynchronize(L->stream));
    L->initialized = true;
    L->step = 0;
    return LB_OK;
}

lb_status lb_init_equilibrium(lb_lattice *L, const double *rho, const double *ux, const double *uy) {
    return lb_init_equilibrium_thermal(L, rho, ux, uy, nullptr);
}

lb_status lb_step(lb_lattice *L, int64_t nsteps) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    if (nsteps < 0) return fail(LB_EINVAL, "negative step count");
    for (int64_t k = 0; k < nsteps; ++k) {
        lb_status st = one_step(L);
        if (st != LB_OK) return st;
    }
    HIPCHK(hipGetLastError());
    return LB_OK;
}

int64_t lb_step_count(const lb_lattice *L) { return L ? L->step : -1; }

lb_status lb_moments(lb_lattice *L, double *rho, double *ux, double *uy, int32_t on_device) {
    if (!L || !rho || !ux || !uy) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    double *o[3] = {rho, ux, uy};
    if (!on_device)
        for (int k = 0; k < 3; ++k) o[k] = L->d_mom + k * N;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.out0 = o[0];
        a.out1 = o[1];
        a.out2 = o[2];
        L->ks[s]->moments(a, node_grid(L), L->stream);
    }
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(rho, o[0], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipMemcpyAsync(ux, o[1], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipMemcpyAsync(uy, o[2], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return LB_OK;
}

lb_status lb_conservation(lb_lattice *L, double out[3]) {
    if (!L || !out) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.out0 = L->d_mom;
        a.out1 = L->d_mom + N;
        a.out2 = L->d_mom + 2 * N;
        L->ks[s]->moments(a, node_grid(L), L->stream);
    }
    const int nb = int(std::min<size_t>(1024, (N + 255) / 256));
    hipLaunchKernelGGL(k_sum3_partial, dim3(nb), dim3(256), 0, L->stream, L->d_mom, L->d_mom + N, L->d_mom + 2 * N,
                       int64_t(N), L->d_part);
    hipLaunchKernelGGL(k_sum3_final, dim3(1), dim3(256), 0, L->stream, L->d_part, nb);
    HIPCHK(hipGetLastError());
    double h[3];
    for (int q = 0; q < 3; ++q)
        HIPCHK(hipMemcpyAsync(&h[q], L->d_part + q * 1024, 8, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    for (int q = 0; q < 3; ++q) out[q] = h[q];
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2]))
        return fail(LB_EUNSTABLE, "non-finite conservation sums after step %lld", (long long)L->step);
    return LB_OK;
}

lb_status lb_thermal_moments(lb_lattice *L, double *T, double *qx, double *qy, int32_t on_device) {
    if (!L || !T || !qx || !qy) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    double *o[3] = {T, qx, qy};
    if (!on_device)
        for (int k = 0; k < 3; ++k) o[k] = L->d_mom + k * N;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.out0 = o[0];
        a.out1 = o[1];
        a.out2 = o[2];
        L->ks[s]->thermal(a, node_grid(L), L->stream);
    }
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(T, o[0], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipMemcpyAsync(qx, o[1], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipMemcpyAsync(qy, o[2], 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return LB_OK;
}

lb_status lb_energy(lb_lattice *L, double *out) {
    if (!L || !out) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.mode = 1;   // energy density into out0
        a.out0 = L->d_mom;
        L->ks[s]->thermal(a, node_grid(L), L->stream);
    }
    // the fixed-order reduction of lb_conservation; its other two sums
    // repeat the first
    const int nb = int(std::min<size_t>(1024, (N + 255) / 256));
    hipLaunchKernelGGL(k_sum3_partial, dim3(nb), dim3(256), 0, L->stream, L->d_mom, L->d_mom, L->d_mom, int64_t(N),
                       L->d_part);
    hipLaunchKernelGGL(k_sum3_final, dim3(1), dim3(256), 0, L->stream, L->d_part, nb);
    HIPCHK(hipGetLastError());
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, L->d_part, 8, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    *out = h;
    if (!std::isfinite(h)) return fail(LB_EUNSTABLE, "non-finite energy after step %lld", (long long)L->step);
    return LB_OK;
}

lb_status lb_get_populations(lb_lattice *L, int32_t which, double *host) {
    if (!L || !host || which < 0 || which > 1) return fail(LB_EINVAL, "bad argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    NodeArgs a = node_args(L, which, L->cur);
    a.out0 = L->d_stage;
    L->ks[which]->get_pop(a, node_grid(L), L->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(host, L->d_stage, 8 * N * L->Q[which], hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    return LB_OK;
}

lb_status lb_set_populations(lb_lattice *L, int32_t which, const double *host) {
    if (!L || !host || which < 0 || which > 1) return fail(LB_EINVAL, "bad argument");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    HIPCHK(hipMemcpyAsync(L->d_stage, host, 8 * N * L->Q[which], hipMemcpyHostToDevice, L->stream));
    NodeArgs a = node_args(L, which, L->cur);
    a.in0 = L->d_stage;
    L->ks[which]->set_pop(a, node_grid(L), L->stream);
    lb_status st = refresh_all(L, 0);
    if (st != LB_OK) return st;
    HIPCHK(hipStreamSynchronize(L->stream));
    L->initialized = true;
    return LB_OK;
}

size_t lb_state_bytes(const lb_lattice *L) {
    if (!L) return 0;
    size_t b = 16;
    for (int s = 0; s < 2; ++s) b += size_t(L->Q[s]) * L->buf[s].plane * esize_of(L->p.storage);
    return b;
}

lb_status lb_get_state(lb_lattice *L, void *host, size_t bytes) {
    if (!L || !host || bytes < lb_state_bytes(L)) return fail(LB_EINVAL, "bad state buffer");
    char *h = reinterpret_cast<char *>(host);
    int64_t hdr[2] = {L->step, L->initialized ? 1 : 0};
    memcpy(h, hdr, 16);
    size_t off = 16;
    for (int s = 0; s < 2; ++s) {
        size_t b = size_t(L->Q[s]) * L->buf[s].plane * esize_of(L->p.storage);
        HIPCHK(hipMemcpyAsync(h + off, L->buf[s].base[L->cur], b, hipMemcpyDeviceToHost, L->stream));
        off += b;
    }
    HIPCHK(hipStreamSynchronize(L->stream));
    return LB_OK;
}

lb_status lb_set_state(lb_lattice *L, const void *host, size_t bytes) {
    if (!L || !host || bytes < lb_state_bytes(L)) return fail(LB_EINVAL, "bad state buffer");
    const char *h = reinterpret_cast<const char *>(host);
    int64_t hdr[2];
    memcpy(hdr, h, 16);
    size_t off = 16;
    for (int s = 0; s < 2; ++s) {
        size_t b = size_t(L->Q[s]) * L->buf[s].plane * esize_of(L->p.storage);
        HIPCHK(hipMemcpyAsync(L->buf[s].base[L->cur], h + off, b, hipMemcpyHostToDevice, L->stream));
        off += b;
    }
    HIPCHK(hipStreamSynchronize(L->stream));
    L->step = hdr[0];
    L->initialized = hdr[1] != 0;
    return LB_OK;
}

lb_status lb_indicator(lb_lattice *L, double *B, int32_t on_device) {
    if (!L || !B) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    const size_t N = size_t(L->p.ny + 1) * L->p.nx;
    double *o = on_device ? B : L->d_mom;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.out0 = o;
        L->ks[s]->indicator(a, node_grid(L), L->stream);
    }
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(B, o, 8 * N, hipMemcpyDeviceToHost, L->stream));
        HIPCHK(hipStreamSynchronize(L->stream));
    }
    return LB_OK;
}

lb_status lb_change_regions(lb_lattice *L, const int32_t *lo, const int32_t *hi) {
    if (!L || !lo || !hi) return fail(LB_EINVAL, "null argument");
    if (!L->initialized) return lb_set_regions(L, lo, hi);
    if (L->p.iface == LB_IFACE_PAPER) return fail(LB_EUNSUPPORTED, "region change with the interpolation interface");
    lb_status st = check_bands(L, lo, hi);
    if (st != LB_OK) return st;
    HIPCHK(hipMemcpyAsync(L->d_oblo, L->d_blo, 4 * L->ntiles, hipMemcpyDeviceToDevice, L->stream));
    HIPCHK(hipMemcpyAsync(L->d_obhi, L->d_bhi, 4 * L->ntiles, hipMemcpyDeviceToDevice, L->stream));
    L->blo.assign(lo, lo + L->ntiles);
    L->bhi.assign(hi, hi + L->ntiles);
    st = upload_regions(L);
    if (st != LB_OK) return st;
    for (int s = 0; s < 2; ++s) {
        NodeArgs a = node_args(L, s, L->cur);
        a.oblo = L->d_oblo;
        a.obhi = L->d_obhi;
        if (L->closure_on) {
            a.clw = L->d_clw;
            a.cn = L->cn;
        }
        L->ks[s]->convert(a, node_grid(L), L->stream);
    }
    st = refresh_all(L, 1);
    if (st != LB_OK) return st;
    if (L->closure_on && L->nproj[0]) {
        // the halo lift of the current copy with the learned closure, as
        // every step does for its new copy
        StepArgs a{};
        a.g = L->geo;
        a.ph = L->ph;
        a.rho_shift = L->rho_shift;
        a.dshift = L->dshift;
        a.cur = L->cur ^ 1;   // the kernels act on copy cur ^ 1
        a.self = L->buf[0];
        a.other = L->buf[1];
        a.items = L->d_proj;
        a.nitems = L->nproj[0];
        a.chunk = 0;
        a.clo = L->d_clo;
        a.clw = L->d_clw;
        a.cn = L->cn;
        L->ks[0]->closure_infer(a, (L->nproj[0] + lbi::CLOSURE_NB - 1) / lbi::CLOSURE_NB, L->stream);
        L->ks[0]->project_halo(a, int((int64_t(L->nproj[0]) * L->n[1] + 127) / 128), L->stream);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(L->stream));
    return LB_OK;
}

lb_status lb_update_regions(lb_lattice *L, double theta, int32_t bmin, int32_t bmax) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (bmin < 0 || bmax < bmin || bmax > L->p.ny / 2) return fail(LB_EINVAL, "bad band limits");
    lb_status st = lb_indicator(L, L->d_mom, 1);
    if (st != LB_OK) return st;
    if (L->closure_on && L->closure_flags) {
        // nodes the network flags count as above any threshold
        NodeArgs a = node_args(L, 0, L->cur);
        a.out0 = L->d_mom;
        a.clw = L->d_clw;
        a.cn = L->cn;
        const int64_t nodes = int64_t(L->p.nx) * (L->p.ny + 1);
        L->ks[0]->closure_flags(a, int((nodes + 15) / 16), L->stream);
        HIPCHK(hipGetLastError());
    }
    int32_t *nlo = L->d_oblo, *nhi = L->d_obhi;   // scratch for the new bands
    hipLaunchKernelGGL(k_bands, dim3(L->ntiles), dim3(256), 0, L->stream, L->d_mom, L->geo, theta, bmin, bmax, nlo,
                       nhi);
    HIPCHK(hipGetLastError());
    std::vector<int32_t> lo(L->ntiles), hi(L->ntiles);
    HIPCHK(hipMemcpyAsync(lo.data(), nlo, 4 * L->ntiles, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipMemcpyAsync(hi.data(), nhi, 4 * L->ntiles, hipMemcpyDeviceToHost, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));
    return lb_change_regions(L, lo.data(), hi.data());
}

lb_status lb_project(int32_t ns, int32_t eqs, int32_t nd, int32_t eqd, const double *f_src, const double *closure,
                     double *f_dst, int64_t n, void *hip_stream) {
    if (!f_src || !f_dst || n < 0) return fail(LB_EINVAL, "bad argument");
    const lbk::KernelSet *k = find_any(ns, eqs, nd, eqd);
    if (!k) return fail(LB_EUNSUPPORTED, "no projection kernel for this pair");
    k->project(f_src, closure, f_dst, n, reinterpret_cast<hipStream_t>(hip_stream));
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_set_closure(lb_lattice *L, const float *params, const float *norm) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (!params) {
        L->closure_on = false;
        L->closure_flags = false;
        return LB_OK;
    }
    if (!norm) return fail(LB_EINVAL, "closure needs its standardisation constants");
    if (L->th) return fail(LB_EUNSUPPORTED, "the learned closure is built for isothermal lattices");
    if (L->n[0] != 3 || L->n[1] != 6 || L->eq[1] != 4)
        return fail(LB_EUNSUPPORTED, "the learned closure is built for D2Q9 lifted to D2Q36 (order 4)");
    for (int k = 0; k < 10; ++k) {
        L->cn.xmean[k] = norm[k];
        L->cn.xstd[k] = norm[10 + k];
    }
    for (int k = 0; k < 6; ++k) {
        L->cn.tmean[k] = norm[20 + k];
        L->cn.tstd[k] = norm[26 + k];
    }
    L->cn.kn_ref = float(L->p.kn);
    L->cn.tau_rho = L->p.tau_mode == LB_TAU_RHO;
    lbk::launch_to_bf16(params, L->d_clw, L->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(L->stream));
    L->closure_on = true;
    return LB_OK;
}

lb_status lb_closure_samples(lb_lattice *L, const int32_t *nodes, int64_t n, double theta, float *x, float *t,
                             int32_t *flag) {
    if (!L || !nodes || !x || !t || !flag || n < 0) return fail(LB_EINVAL, "bad argument");
    if (!L->initialized) return fail(LB_ESTATE, "lattice not initialised");
    if (L->n[0] != 3 || L->n[1] != 6) return fail(LB_EUNSUPPORTED, "samples are drawn for the D2Q9/D2Q36 pair");
    if (L->th) return fail(LB_EUNSUPPORTED, "samples are drawn from isothermal lattices");
    NodeArgs a = node_args(L, 1, L->cur);
    a.nodes = nodes;
    a.nnodes = n;
    a.theta = theta;
    a.fx = x;
    a.ft = t;
    a.flag = flag;
    if (n) L->ks[1]->closure_samples(a, int((n + 63) / 64), L->stream);
    HIPCHK(hipGetLastError());
    return LB_OK;
}

lb_status lb_set_closure_flags(lb_lattice *L, int32_t enable) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (enable && !L->closure_on) return fail(LB_ESTATE, "set the learned closure first (lb_set_closure)");
    L->closure_flags = enable != 0;
    return LB_OK;
}

lb_status lb_set_merged_update(lb_lattice *L, int32_t enable) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (!enable && d2q9_alone_off(L))
        return fail(LB_EUNSUPPORTED, "thermal lattices with a D2Q9 low set use the merged update");
    L->merged = enable != 0;
    return LB_OK;
}

lb_status lb_set_concurrency(lb_lattice *L, int32_t enable) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (enable && d2q9_alone_off(L))
        return fail(LB_EUNSUPPORTED, "thermal lattices with a D2Q9 low set use the merged update");
    L->concurrent = enable != 0;
    return LB_OK;
}

lb_status lb_set_timing(lb_lattice *L, int32_t enable) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    if (enable < 0) return fail(LB_EINVAL, "timing takes 0 (off) or a step interval >= 1");
    HIPCHK(hipStreamSynchronize(L->stream));
    L->timing = enable != 0;
    L->timing_every = enable > 0 ? enable : 1;
    L->ev_used = 0;
    L->ev_kind.clear();
    return LB_OK;
}

lb_status lb_kernel_times(lb_lattice *L, double *ms_high, int64_t *n_high, double *ms_all, int64_t *n_all) {
    if (!L) return fail(LB_EINVAL, "null lattice");
    HIPCHK(hipStreamSynchronize(L->stream));
    double mh = 0, ma = 0;
    int64_t nh = 0, na = 0;
    for (size_t k = 0; k < L->ev_kind.size(); ++k) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, L->ev_pool[2 * k], L->ev_pool[2 * k + 1]));
        ma += ms;
        na++;
        if (L->ev_kind[k] == L->dom) {
            mh += ms;
            nh++;
        }
    }
    if (ms_high) *ms_high = mh;
    if (n_high) *n_high = nh;
    if (ms_all) *ms_all = ma;
    if (n_all) *n_all = na;
    L->ev_used = 0;
    L->ev_kind.clear();
    return LB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
// Many independent lattices stepped together: per step, one update launch
// covers the work items of every lattice and velocity set, and one
// projection launch every set pair (each item names its lattice, whose
// arguments sit in a device descriptor table), all on one stream,
// optionally replayed from a captured HIP graph.

struct lb_batch {
    struct Kind {
        const lbk::KernelSet *ks[2];   // the pair's kernels, self = low / high set
        std::vector<int> members;      // lattice indices
        int32_t *d_fin = nullptr;
        int nfin = 0;
        int32_t *d_proj = nullptr;
        int nup = 0, ndown = 0;
        bool merged = false;           // projected by a merged launch (else by one of its own)
    };
    std::vector<lb_lattice *> lat;
    std::vector<int64_t> gen;          // region generation of each lattice at the last build
    // update work items grouped by velocity set: the update of a set does
    // not depend on its partner, so one launch serves the set in every pair
    struct SetGroup {
        int n, eq;
        int32_t *d_items = nullptr;    // (i0, j0, j1, side * nlat + lattice)
        int nitems = 0, chunk = 0;
    };
    std::vector<Kind> kinds;
    std::vector<SetGroup> groups;
    // merged launches: per registered kernel pair, the groups in its update
    // slots (D2Q36, D2Q16, D2Q9) and the kinds in its projection slots
    // (D2Q9/D2Q36, D2Q16/D2Q36, D2Q9/D2Q16), -1 where empty
    struct Plan {
        const lbk::MultiSet *ms;
        int group[3];
        int kind[3];
    };
    std::vector<Plan> plans;
    lbk::Registry reg;
    hipStream_t stream;
    StepArgs *d_desc[2];               // per lattice, self = low set / high set (one allocation, high after low)
    int strip[2];                      // rows per work item (0 = automatic)
    int cur;
    int seg;                           // steps per captured graph (0 = direct launches)
    hipGraph_t graph[2];               // one per starting copy parity
    hipGraphExec_t exec[2];
    hipEvent_t ev, t0, t1;
    int64_t nodes;
    // persistent launches (lb_batch_set_persistent): per-workgroup lattice
    // lists, per-lattice item and projection ranges
    bool persistent = false;
    const lbk::MultiSet *pms = nullptr;
    int32_t *d_pwl_off = nullptr, *d_pwl = nullptr, *d_plat = nullptr, *d_pitems = nullptr, *d_pproj = nullptr;
    int pgrid = 0;
};

namespace {

lb_status upload_list(const std::vector<int32_t> &v, int32_t *&d, hipStream_t s) {
    if (d) {
        HIPCHK(hipFree(d));
        d = nullptr;
    }
    if (v.empty()) return LB_OK;
    HIPCHK(hipMalloc(&d, v.size() * 4));
    HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * 4, hipMemcpyHostToDevice, s));
    return LB_OK;
}

void batch_drop_graphs(lb_batch *B) {
    for (int p = 0; p < 2; ++p) {
        if (B->exec[p]) (void)hipGraphExecDestroy(B->exec[p]);
        if (B->graph[p]) (void)hipGraphDestroy(B->graph[p]);
        B->exec[p] = nullptr;
        B->graph[p] = nullptr;
    }
}

// Lists of the persistent launch: every lattice's update items (one wave
// each, D2Q36 first) and projection entries, and the workgroups' lattices,
// assigned largest-first (populations x nodes) to the least loaded of
// min(lattices, CUs) workgroups.
lb_status persist_build(lb_batch *B) {
    const int nl = int(B->lat.size());
    B->pms = nullptr;
    for (int m = 0; m < B->reg.nmulti && !B->pms; ++m) {
        const lbk::MultiSet &ms = B->reg.multi[m];
        bool ok = ms.persist != nullptr;
        for (lb_lattice *L : B->lat)
            for (int s = 0; s < 2; ++s) {
                const int n = L->n[s], e = L->eq[s];
                ok = ok && ((n == 6 && e == ms.eq6) || (n == 4 && e == ms.eq4) || (n == 3 && e == 2));
            }
        if (ok) B->pms = &ms;
    }
    if (!B->pms) return fail(LB_EUNSUPPORTED, "no persistent batch kernel for these velocity sets and orders");
    std::vector<int32_t> items, proj, lat(size_t(8) * nl, 0), f1, p1;
    std::vector<std::pair<int, int>> runs;
    std::vector<int> runcol;
    std::vector<double> cost(nl, 0.0);
    for (int l = 0; l < nl; ++l) {
        lb_lattice *L = B->lat[l];
        int np[2];
        const int nfin = build_lists(L, f1, p1, np);
        if (nfin) return fail(LB_EUNSUPPORTED, "lattice %d needs a finish pass (periodic rows or pressure columns): "
                                               "not in persistent launches", l);
        if (L->n[0] == L->n[1] && np[0] + np[1])
            return fail(LB_EUNSUPPORTED, "lattice %d: equal sets with bands are not in persistent launches", l);
        lat[8 * l] = int32_t(items.size() / 4);
        const bool wrap = L->p.nx == 8 && L->p.xbc == LB_XBC_PERIODIC;
        const int ng = wrap ? 8 : 64 / (L->p.nx + 4);
        // the high (heavier) set's items first, so that waves start with them
        for (int s : {1, 0}) {
            const int kind = L->n[s] == 6 ? 0 : L->n[s] == 4 ? 1 : 2;
            const int strip = B->strip[s] > 0 ? B->strip[s] : 4;
            const int span = ng >= 2 ? ng * strip : strip;
            set_runs(L, s, runs, runcol);
            for (size_t r = 0; r < runs.size(); ++r)
                for (int j = runs[r].first; j < runs[r].second; j += span) {
                    items.insert(items.end(), {wrap ? -(strip + lbi::NW_WRAP) : ng >= 2 ? -strip : runcol[r], j,
                                               std::min(j + span, runs[r].second), (s * nl + l) | (kind << 28)});
                    cost[l] += double(L->Q[s]) * (std::min(j + span, runs[r].second) - j) *
                               (ng >= 2 ? L->p.nx : 60);
                }
        }
        lat[8 * l + 1] = int32_t(items.size() / 4) - lat[8 * l];
        lat[8 * l + 2] = int32_t(proj.size() / 4);
        for (int e = 0; e < np[0] + np[1]; ++e) proj.insert(proj.end(), {p1[2 * e], p1[2 * e + 1], l, 0});
        lat[8 * l + 3] = np[0];
        lat[8 * l + 4] = np[1];
        const int nlo = L->n[0], nhi = L->n[1];
        lat[8 * l + 5] = nhi == 6 ? (nlo == 3 ? 0 : 1) : 2;
    }
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int nwg = std::max(1, std::min(nl, cus));
    std::vector<int> order(nl);
    for (int l = 0; l < nl; ++l) order[l] = l;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(nwg, 0.0);
    std::vector<std::vector<int32_t>> own(nwg);
    for (int l : order) {
        const int g = int(std::min_element(load.begin(), load.end()) - load.begin());
        load[g] += cost[l];
        own[g].push_back(l);
    }
    std::vector<int32_t> off(1, 0), wl;
    for (auto &o : own) {
        wl.insert(wl.end(), o.begin(), o.end());
        off.push_back(int32_t(wl.size()));
    }
    lb_status st = upload_list(off, B->d_pwl_off, B->stream);
    if (st == LB_OK) st = upload_list(wl, B->d_pwl, B->stream);
    if (st == LB_OK) st = upload_list(lat, B->d_plat, B->stream);
    if (st == LB_OK) st = upload_list(items, B->d_pitems, B->stream);
    if (st == LB_OK) st = upload_list(proj.empty() ? std::vector<int32_t>(4, 0) : proj, B->d_pproj, B->stream);
    if (st != LB_OK) return st;
    B->pgrid = nwg;
    return LB_OK;
}

// merged work lists of every pair kind
lb_status batch_build(lb_batch *B) {
    batch_drop_graphs(B);
    std::vector<std::pair<int, int>> runs;
    std::vector<int> runcol;
    const int nl = int(B->lat.size());
    std::vector<std::vector<int32_t>> gv(B->groups.size());
    for (auto &K : B->kinds) {
        for (int s = 0; s < 2; ++s) {
            size_t g = 0;
            while (g < B->groups.size() && !(B->groups[g].n == K.ks[s]->nS && B->groups[g].eq == K.ks[s]->eqS)) ++g;
            int64_t rows = 0;
            for (int l : K.members) rows += set_runs(B->lat[l], s, runs, runcol);
            const int strip = B->strip[s] > 0 ? B->strip[s] : auto_strip(rows);
            // items ordered by lattice, column group and row (cut into XCD
            // slabs below) so neighbouring strips of one lattice share an L2
            std::vector<int32_t> &v = gv[g];
            for (int l : K.members) {
                set_runs(B->lat[l], s, runs, runcol);
                // a lattice at most 28 columns wide packs 64 / (nx + 4) lane
                // groups into a wave, each marching `strip` rows of its own;
                // such items carry -strip as their first column.  An
                // 8-column periodic lattice takes 8 groups of 8 lanes with
                // the x neighbours wrapped in the group: -(strip + NW_WRAP)
                const lb_lattice *La = B->lat[l];
                const bool wrap = La->p.nx == 8 && La->p.xbc == LB_XBC_PERIODIC;
                const int ng = wrap ? 8 : 64 / (La->p.nx + 4);
                const int span = ng >= 2 ? ng * strip : strip;
                for (size_t r = 0; r < runs.size(); ++r)
                    for (int j = runs[r].first; j < runs[r].second; j += span) {
                        v.push_back(wrap ? -(strip + lbi::NW_WRAP) : ng >= 2 ? -strip : runcol[r]);
                        v.push_back(j);
                        v.push_back(std::min(j + span, runs[r].second));
                        v.push_back(s * nl + l);
                    }
            }
        }
    }
    for (size_t g = 0; g < B->groups.size(); ++g) {
        auto &G = B->groups[g];
        std::vector<int32_t> &v = gv[g];
        const int n = int(v.size() / 4);
        G.chunk = (n + 7) / 8;   // 8 contiguous slabs, one per XCD through the kernel's mapping
        v.resize(size_t(8) * G.chunk * 4, 0);   // padding items are empty (j0 = j1)
        G.nitems = 8 * G.chunk;
        lb_status st = upload_list(v, G.d_items, B->stream);
        if (st != LB_OK) return st;
    }
    for (auto &K : B->kinds) {
        std::vector<int32_t> fin, up, down, f1, p1;
        for (int l : K.members) {
            lb_lattice *L = B->lat[l];
            int np[2];
            build_lists(L, f1, p1, np);
            for (size_t k = 0; k < f1.size(); k += 4) {
                fin.insert(fin.end(), {f1[k], f1[k + 1], f1[k + 2], l});
            }
            for (int e = 0; e < np[0] + np[1]; ++e) {
                std::vector<int32_t> &d = e < np[0] ? up : down;
                d.insert(d.end(), {p1[2 * e], p1[2 * e + 1], l, 0});
            }
        }
        K.nfin = int(fin.size() / 4);
        K.nup = int(up.size() / 4);
        K.ndown = int(down.size() / 4);
        up.insert(up.end(), down.begin(), down.end());
        lb_status st = upload_list(fin, K.d_fin, B->stream);
        if (st == LB_OK) st = upload_list(up, K.d_proj, B->stream);
        if (st != LB_OK) return st;
    }
    // merged launches: each set group takes its slot in the first registered
    // kernel pair that has one for it; a kind's projection goes to a merged
    // launch when its set pair is one of the projection slots, else to a
    // launch of its own
    B->plans.clear();
    for (auto &K : B->kinds) K.merged = false;
    std::vector<char> placed(B->groups.size(), 0);
    for (int m = 0; m < B->reg.nmulti; ++m) {
        const lbk::MultiSet &ms = B->reg.multi[m];
        const int sn[3] = {6, 4, 3}, se[3] = {ms.eq6, ms.eq4, 2};
        lb_batch::Plan P{&ms, {-1, -1, -1}, {-1, -1, -1}};
        bool any = false;
        for (int s = 0; s < 3; ++s)
            for (size_t g = 0; g < B->groups.size(); ++g)
                if (!placed[g] && B->groups[g].n == sn[s] && B->groups[g].eq == se[s]) {
                    placed[g] = 1;
                    if (B->groups[g].chunk) {
                        P.group[s] = int(g);
                        any = true;
                    }
                }
        for (size_t k = 0; k < B->kinds.size(); ++k) {
            auto &K = B->kinds[k];
            if (K.nup + K.ndown == 0 || K.merged) continue;
            const int nl = K.ks[0]->nS, el = K.ks[0]->eqS, nh = K.ks[1]->nS, eh = K.ks[1]->eqS;
            int s = -1;
            if (nl == 3 && el == 2 && nh == 6 && eh == ms.eq6) s = 0;
            else if (nl == 4 && el == ms.eq4 && nh == 6 && eh == ms.eq6) s = 1;
            else if (nl == 3 && el == 2 && nh == 4 && eh == ms.eq4) s = 2;
            if (s < 0) continue;
            P.kind[s] = int(k);
            K.merged = true;
            any = true;
        }
        if (any) B->plans.push_back(P);
    }
    for (size_t g = 0; g < B->groups.size(); ++g)
        if (!placed[g])
            return fail(LB_EUNSUPPORTED, "no batched update kernel for D2Q%d of order %d in this storage",
                        B->groups[g].n * B->groups[g].n, B->groups[g].eq);
    if (B->persistent) {
        lb_status st = persist_build(B);
        if (st != LB_OK) return st;
    }
    HIPCHK(hipStreamSynchronize(B->stream));
    for (size_t l = 0; l < B->lat.size(); ++l) B->gen[l] = B->lat[l]->gen;
    return LB_OK;
}

// the launches of one step of every lattice (source copy cur), in stream
// order: the merged update launches, then the merged projection launches
// (and those of set pairs outside their slots), then the finish passes
lb_status batch_launch(lb_batch *B, int cur, uint32_t seed) {
    for (auto &P : B->plans) {
        BatchMulti m{};
        m.desc = B->d_desc[0];
        m.cur = cur;
        m.seed = seed;
        int nb = 0;
        for (int s = 0; s < 3; ++s) {
            m.start[s] = nb;
            if (P.group[s] < 0) continue;
            const auto &G = B->groups[P.group[s]];
            m.items[s] = G.d_items;
            m.nitems[s] = G.nitems;
            m.nsplit[s] = G.chunk;
            // D2Q36 / D2Q16: a block per item; D2Q9: one item per wave
            const int W = P.ms->waves;
            nb += 8 * (s < 2 ? G.chunk : (G.chunk + W - 1) / W);
        }
        m.start[3] = nb;
        if (nb) P.ms->update(m, nb, B->stream);
    }
    for (auto &P : B->plans) {
        BatchMulti m{};
        m.desc = B->d_desc[0];
        m.cur = cur;
        m.seed = seed;
        int nb = 0;
        for (int s = 0; s < 3; ++s) {
            m.start[s] = nb;
            if (P.kind[s] < 0) continue;
            const auto &K = B->kinds[P.kind[s]];
            m.items[s] = K.d_proj;
            m.nitems[s] = K.nup;
            m.nsplit[s] = K.ndown;
            // one thread per (node, target column)
            const int64_t nt = int64_t(K.nup) * K.ks[1]->nS + int64_t(K.ndown) * K.ks[0]->nS;
            nb += int((nt + 127) / 128);
        }
        m.start[3] = nb;
        if (nb) P.ms->project(m, nb, B->stream);
    }
    for (auto &K : B->kinds) {
        if (K.merged || !(K.nup + K.ndown)) continue;
        const int64_t nt = int64_t(K.nup) * K.ks[1]->nS + int64_t(K.ndown) * K.ks[0]->nS;
        BatchArgs a{B->d_desc[0], K.d_proj, K.nup, 0, cur, K.ndown, seed};
        K.ks[0]->project_batch(a, int((nt + 127) / 128), B->stream);
    }
    for (auto &K : B->kinds) {
        if (!K.nfin) continue;
        BatchArgs a{B->d_desc[0], K.d_fin, K.nfin, 0, cur, 0, seed};
        const int qm = std::max(K.ks[0]->nS * K.ks[0]->nS, K.ks[1]->nS * K.ks[1]->nS);
        K.ks[0]->finish_batch(a, int((int64_t(K.nfin) * qm + 127) / 128), B->stream);
    }
    return LB_OK;
}

// n steps of every lattice from copy B->cur, step numbers from step0: one
// set of launches per step, or persistent launches of up to 4096 steps
lb_status batch_steps(lb_batch *B, int64_t n, int64_t step0) {
    int64_t k = 0;
    while (k < n) {
        if (B->persistent) {
            PersistArgs a{};
            a.desc = B->d_desc[0];
            a.wl_off = B->d_pwl_off;
            a.wl = B->d_pwl;
            a.lat = B->d_plat;
            a.items = B->d_pitems;
            a.proj = B->d_pproj;
            a.nsteps = int32_t(std::min<int64_t>(4096, n - k));
            a.cur = B->cur;
            a.step0 = step0 + k;
            B->pms->persist(a, B->pgrid, B->stream);
            B->cur ^= a.nsteps & 1;
            k += a.nsteps;
        } else {
            lb_status st = batch_launch(B, B->cur, step_seed(step0 + k));
            if (st != LB_OK) return st;
            B->cur ^= 1;
            ++k;
        }
    }
    return LB_OK;
}

lb_status batch_check(lb_batch *B) {
    bool stale = false;
    for (size_t l = 0; l < B->lat.size(); ++l) {
        lb_lattice *L = B->lat[l];
        if (L->cur != B->cur) return fail(LB_ESTATE, "lattice %zu was stepped outside the batch (copy parity)", l);
        if (L->closure_on) return fail(LB_EUNSUPPORTED, "lattice %zu uses the learned closure", l);
        if (L->gen != B->gen[l]) stale = true;
    }
    return stale ? batch_build(B) : LB_OK;
}

// order the batch stream after (into = true) or before the lattices' streams
lb_status batch_join(lb_batch *B, bool into) {
    std::vector<hipStream_t> seen;
    for (lb_lattice *L : B->lat) {
        if (L->stream == B->stream || std::find(seen.begin(), seen.end(), L->stream) != seen.end()) continue;
        seen.push_back(L->stream);
        if (into) {
            HIPCHK(hipEventRecord(B->ev, L->stream));
            HIPCHK(hipStreamWaitEvent(B->stream, B->ev, 0));
        } else {
            HIPCHK(hipEventRecord(B->ev, B->stream));
            HIPCHK(hipStreamWaitEvent(L->stream, B->ev, 0));
        }
    }
    return LB_OK;
}

lb_status batch_run(lb_batch *B, int64_t steps) {
    int64_t k = 0;
    if (B->seg > 0) {
        while (steps - k >= B->seg) {
            const int par = B->cur;
            if (!B->exec[par]) {
                HIPCHK(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
                // (a replayed graph repeats its segment's seeds)
                lb_status st = batch_steps(B, B->seg, B->lat[0]->step + k);
                B->cur = par;
                hipGraph_t g = nullptr;
                hipError_t e = hipStreamEndCapture(B->stream, &g);
                if (st != LB_OK) {
                    if (g) (void)hipGraphDestroy(g);
                    return st;
                }
                if (e != hipSuccess || !g) return fail(LB_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
                B->graph[par] = g;
                HIPCHK(hipGraphInstantiate(&B->exec[par], g, nullptr, nullptr, 0));
            }
            HIPCHK(hipGraphLaunch(B->exec[par], B->stream));
            B->cur ^= B->seg & 1;
            k += B->seg;
        }
    }
    if (k < steps) {
        lb_status st = batch_steps(B, steps - k, B->lat[0]->step + k);
        if (st != LB_OK) return st;
    }
    HIPCHK(hipGetLastError());
    for (lb_lattice *L : B->lat) {
        L->cur = B->cur;
        L->step += steps;
    }
    return LB_OK;
}

}  // namespace

extern "C" {

lb_status lb_batch_create(lb_lattice *const *lattices, int32_t n, void *hip_stream, lb_batch **out) {
    if (!lattices || n < 1 || !out) return fail(LB_EINVAL, "bad argument");
    *out = nullptr;
    const int cur = lattices[0] ? lattices[0]->cur : 0;
    for (int l = 0; l < n; ++l) {
        const lb_lattice *L = lattices[l];
        if (!L) return fail(LB_EINVAL, "null lattice %d", l);
        if (!L->initialized) return fail(LB_ESTATE, "lattice %d not initialised", l);
        if (L->p.storage != lattices[0]->p.storage) return fail(LB_EINVAL, "lattices of one batch share a storage type");
        if (L->p.iface != LB_IFACE_HERMITE) return fail(LB_EUNSUPPORTED, "batches use the Hermite interface");
        if (L->closure_on) return fail(LB_EUNSUPPORTED, "lattice %d uses the learned closure", l);
        if (L->th) return fail(LB_EUNSUPPORTED, "lattice %d is thermal (batches are isothermal)", l);
        if (L->p.u_osc != 0.0) return fail(LB_EUNSUPPORTED, "lattice %d has an oscillating wall", l);
        if (L->cur != cur) return fail(LB_ESTATE, "lattices of one batch must be at the same copy parity");
        for (int m = 0; m < l; ++m)
            if (lattices[m] == L) return fail(LB_EINVAL, "lattice %d listed twice", l);
    }
    lb_batch *B = new lb_batch();
    B->lat.assign(lattices, lattices + n);
    B->gen.assign(n, -1);
    B->stream = reinterpret_cast<hipStream_t>(hip_stream);
    B->strip[0] = B->strip[1] = 0;
    B->cur = cur;
    B->seg = 0;
    B->graph[0] = B->graph[1] = nullptr;
    B->exec[0] = B->exec[1] = nullptr;
    B->d_desc[0] = B->d_desc[1] = nullptr;
    B->ev = B->t0 = B->t1 = nullptr;
    B->nodes = 0;
    B->reg = lattices[0]->p.storage == LB_STORE_F64   ? lbk::registry_f64()
             : lattices[0]->p.storage == LB_STORE_F32 ? lbk::registry_f32()
                                                       : lbk::registry_bf16();
    auto bail = [&](lb_status st) {
        lb_batch_destroy(B);
        return st;
    };
    std::vector<StepArgs> desc[2];
    for (int l = 0; l < n; ++l) {
        lb_lattice *L = B->lat[l];
        B->nodes += int64_t(L->p.nx) * (L->p.ny + 1);
        for (int s = 0; s < 2; ++s) {
            StepArgs a{};
            a.g = L->geo;
            a.ph = L->ph;
            a.rho_shift = L->rho_shift;
            a.dshift = L->dshift;
            a.self = L->buf[s];
            a.other = L->buf[1 - s];
            a.ks = L->kconst[s];
            a.self_high = s;
            desc[s].push_back(a);
        }
        size_t k = 0;
        while (k < B->kinds.size() && B->kinds[k].ks[0] != L->ks[0]) ++k;
        if (k == B->kinds.size()) {
            lb_batch::Kind K;
            K.ks[0] = L->ks[0];
            K.ks[1] = L->ks[1];
            B->kinds.push_back(K);
        }
        B->kinds[k].members.push_back(l);
        for (int s = 0; s < 2; ++s) {
            size_t g = 0;
            while (g < B->groups.size() && !(B->groups[g].n == L->ks[s]->nS && B->groups[g].eq == L->ks[s]->eqS)) ++g;
            if (g == B->groups.size()) {
                lb_batch::SetGroup G;
                G.n = L->ks[s]->nS;
                G.eq = L->ks[s]->eqS;
                B->groups.push_back(G);
            }
        }
    }
    if (hipMalloc(&B->d_desc[0], sizeof(StepArgs) * 2 * n) != hipSuccess) return bail(fail(LB_ENOMEM, "descriptor table"));
    B->d_desc[1] = B->d_desc[0] + n;
    for (int s = 0; s < 2; ++s)
        if (hipMemcpy(B->d_desc[s], desc[s].data(), sizeof(StepArgs) * n, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(LB_EDEVICE, "descriptor upload failed"));
    if (hipEventCreateWithFlags(&B->ev, hipEventDisableTiming) != hipSuccess || hipEventCreate(&B->t0) != hipSuccess ||
        hipEventCreate(&B->t1) != hipSuccess)
        return bail(fail(LB_EDEVICE, "event creation failed"));
    lb_status st = batch_build(B);
    if (st != LB_OK) return bail(st);
    *out = B;
    return LB_OK;
}

void lb_batch_destroy(lb_batch *B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    else (void)hipDeviceSynchronize();
    batch_drop_graphs(B);
    for (auto &K : B->kinds) {
        if (K.d_fin) (void)hipFree(K.d_fin);
        if (K.d_proj) (void)hipFree(K.d_proj);
    }
    for (auto &G : B->groups)
        if (G.d_items) (void)hipFree(G.d_items);
    for (int32_t *p : {B->d_pwl_off, B->d_pwl, B->d_plat, B->d_pitems, B->d_pproj})
        if (p) (void)hipFree(p);
    if (B->d_desc[0]) (void)hipFree(B->d_desc[0]);
    if (B->ev) (void)hipEventDestroy(B->ev);
    if (B->t0) (void)hipEventDestroy(B->t0);
    if (B->t1) (void)hipEventDestroy(B->t1);
    delete B;
}

lb_status lb_batch_set_persistent(lb_batch *B, int32_t enable) {
    if (!B) return fail(LB_EINVAL, "null batch");
    const bool on = enable != 0;
    if (on == B->persistent) return LB_OK;
    B->persistent = on;
    lb_status st = batch_build(B);
    if (st != LB_OK) {
        B->persistent = false;
        lb_status st2 = batch_build(B);
        return st2 != LB_OK ? st2 : st;
    }
    return LB_OK;
}

lb_status lb_batch_set_graph(lb_batch *B, int32_t segment_steps) {
    if (!B || segment_steps < 0) return fail(LB_EINVAL, "bad argument");
    if (segment_steps > 0 && !B->stream) return fail(LB_EINVAL, "graph capture needs a created (non-null) stream");
    if (segment_steps != B->seg) batch_drop_graphs(B);
    B->seg = segment_steps;
    return LB_OK;
}

lb_status lb_batch_set_strip_rows(lb_batch *B, int32_t rows_low, int32_t rows_high) {
    if (!B || rows_low < 0 || rows_high < 0) return fail(LB_EINVAL, "bad argument");
    B->strip[0] = rows_low;
    B->strip[1] = rows_high;
    return batch_build(B);
}

lb_status lb_batch_step(lb_batch *B, int64_t steps) {
    if (!B || steps < 0) return fail(LB_EINVAL, "bad argument");
    lb_status st = batch_check(B);
    if (st == LB_OK) st = batch_join(B, true);
    if (st == LB_OK) st = batch_run(B, steps);
    if (st == LB_OK) st = batch_join(B, false);
    return st;
}

lb_status lb_batch_autotune(lb_batch *B, int32_t steps, int32_t rows_out[2]) {
    if (!B || steps < 1) return fail(LB_EINVAL, "bad argument");
    lb_status st = batch_check(B);
    if (st != LB_OK) return st;
    // the trials advance the lattices: keep their states and restore them
    std::vector<std::vector<char>> saved(B->lat.size());
    for (size_t l = 0; l < B->lat.size(); ++l) {
        saved[l].resize(lb_state_bytes(B->lat[l]));
        if ((st = lb_get_state(B->lat[l], saved[l].data(), saved[l].size())) != LB_OK) return st;
    }
    const int cur0 = B->cur, seg0 = B->seg;
    B->seg = 0;
    static const int cand[] = {1, 2, 4, 8, 16, 32, 64};
    if ((st = batch_join(B, true)) != LB_OK) return st;
    for (int s = 0; s < 2; ++s) {
        double best = 1e300;
        int best_rows = 1;
        for (int c : cand) {
            B->strip[s] = c;
            if ((st = batch_build(B)) != LB_OK) return st;
            // timed twice, the faster pass counting
            for (int rep = 0; rep < 2; ++rep) {
                HIPCHK(hipEventRecord(B->t0, B->stream));
                if ((st = batch_steps(B, steps, 0)) != LB_OK) return st;
                HIPCHK(hipEventRecord(B->t1, B->stream));
                HIPCHK(hipEventSynchronize(B->t1));
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, B->t0, B->t1));
                if (ms < best) {
                    best = ms;
                    best_rows = c;
                }
            }
        }
        B->strip[s] = best_rows;
    }
    if ((st = batch_build(B)) != LB_OK) return st;
    B->cur = cur0;
    B->seg = seg0;
    for (size_t l = 0; l < B->lat.size(); ++l) {
        lb_lattice *L = B->lat[l];
        L->cur = cur0;
        if ((st = lb_set_state(L, saved[l].data(), saved[l].size())) != LB_OK) return st;
    }
    if (rows_out) {
        rows_out[0] = B->strip[0];
        rows_out[1] = B->strip[1];
    }
    return LB_OK;
}

lb_status lb_batch_info(const lb_batch *B, int64_t *nodes, int32_t *launches_per_step, int32_t *kinds) {
    if (!B) return fail(LB_EINVAL, "null batch");
    int nl = 0;
    for (auto &P : B->plans) {
        bool up = false, pr = false;
        for (int s = 0; s < 3; ++s) {
            up = up || P.group[s] >= 0;
            pr = pr || P.kind[s] >= 0;
        }
        nl += up + pr;
    }
    for (auto &K : B->kinds) nl += (!K.merged && K.nup + K.ndown > 0) + (K.nfin > 0);
    if (nodes) *nodes = B->nodes;
    if (launches_per_step) *launches_per_step = B->persistent ? 0 : nl;
    if (kinds) *kinds = int32_t(B->kinds.size());
    return LB_OK;
}

}  // extern "C"

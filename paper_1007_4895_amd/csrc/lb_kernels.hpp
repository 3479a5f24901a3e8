// lb_kernels.hpp -- HIP kernels for gfx950 (CDNA4, wave64).
//
// The hot kernel, k_update, advances every node of one velocity set by one
// time step of Sec. 3.1:
//   f^{n+1} = f - nu_x [F_{i+1/2} - F_{i-1/2}] - nu_y [F_{j+1/2} - F_{j-1/2}]
//             + (dt / tau)(f_eq - f) + dt g,
// with the TVD/minmod face values of Sec. 3.1, the order-N Hermite
// equilibrium of Eq. (approxfeq) and the Hermite body force (Sec. 2.1).
//
// Mapping: a work item is 60 consecutive columns x a strip of rows; its
// waves load 64 columns (two halo columns on each side) and each lane
// marches up one column keeping, per population, the values and limited
// slopes it needs along y in registers, so every population value is loaded
// from HBM once per strip.  The x neighbours come from the neighbouring
// lanes through DPP wave shifts.  The minmod limited slope
// Delta+ Psi(Delta-/Delta+) is evaluated as med3(Delta-, Delta+, 0), which
// is the same function.  Diffuse walls (Sec. 3.2), wall ghost rows and
// periodic image columns are written by the kernel that updates the node.
//
// Nodes with other duties -- periodic row images, pressure columns
// (k_finish), and nodes that a stencil of the partner set reads (Hermite
// projection, Sec. 2.2 in moment form: k_project_halo) -- are finished by
// node-local FP64 passes over lists of those nodes, one launch for both
// (k_project_finish) when a lattice has both lists, so that the hot kernel
// carries none of that register footprint.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lb_internal.hpp"
#include "lb_tables.hpp"

// waves per block of the D2Q36 update (each evolves 6 / LB_SPLIT36 of the
// y-abscissae) and the occupancy it is compiled for, on its own and merged
// with D2Q9 items or in a batch (measured best: 5 and 4 waves per SIMD)
#ifndef LB_SPLIT36
#define LB_SPLIT36 3
#endif
#ifndef LB_WAVES36
#define LB_WAVES36 5
#endif
#ifndef LB_WAVES36_PAIR
#define LB_WAVES36_PAIR 4
#endif
// waves per D2Q36 item in the merged launch with D2Q9 (measured best: 2)
#ifndef LB_PAIR_SPLIT36
#define LB_PAIR_SPLIT36 2
#endif
// row offset in the vector offset of every buffer access (the scalar offset
// then holds the population plane alone, loop-invariant), or in the scalar
// offset for wide items
#ifndef LB_ROWV
#define LB_ROWV 1
#endif
// the batch update of every set in one launch: waves per D2Q36 and D2Q16
// item, and the occupancy it is compiled for
#ifndef LB_MULTI_SPLIT36
#define LB_MULTI_SPLIT36 3
#endif
#ifndef LB_MULTI_SPLIT16
#define LB_MULTI_SPLIT16 2
#endif
#ifndef LB_MULTI_WAVES
#define LB_MULTI_WAVES LB_WAVES36_PAIR
#endif

namespace lbk {

using namespace lbi;
using lbt::NoSet;
using lbt::VSet;

// ------------------------------------------------------------------ storage
struct StF64 {
    using S = double;
    using M = double;
    static constexpr int bytes = 8;
    __device__ static __forceinline__ M ld(const S *p) { return *p; }
    __device__ static __forceinline__ void st(S *p, M v) { *p = v; }
    __device__ static __forceinline__ double ldd(const S *p) { return *p; }
    __device__ static __forceinline__ void std_(S *p, double v) { *p = v; }
    __device__ static __forceinline__ M bld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    __device__ static __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                              r, vo, so, 0);
    }
    static constexpr bool kSR = false;
    __device__ static __forceinline__ void bst_r(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v, uint32_t) {
        bst(r, vo, so, v);
    }
};

struct StF32 {
    using S = float;
    using M = float;
    static constexpr int bytes = 4;
    __device__ static __forceinline__ M ld(const S *p) { return *p; }
    __device__ static __forceinline__ void st(S *p, M v) { *p = v; }
    __device__ static __forceinline__ double ldd(const S *p) { return double(*p); }
    __device__ static __forceinline__ void std_(S *p, double v) { *p = float(v); }
    __device__ static __forceinline__ M bld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    __device__ static __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
    }
    static constexpr bool kSR = false;
    __device__ static __forceinline__ void bst_r(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v, uint32_t) {
        bst(r, vo, so, v);
    }
};

// bfloat16 bits; round to nearest even on store
struct StBF16 {
    using S = uint16_t;
    using M = float;
    static constexpr int bytes = 2;
    __device__ static __forceinline__ float cvt(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
    __device__ static __forceinline__ uint16_t rne(float v) {
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return uint16_t(u >> 16);
    }
    __device__ static __forceinline__ M ld(const S *p) { return cvt(*p); }
    __device__ static __forceinline__ void st(S *p, M v) { *p = rne(v); }
    __device__ static __forceinline__ double ldd(const S *p) { return double(cvt(*p)); }
    __device__ static __forceinline__ void std_(S *p, double v) { *p = rne(float(v)); }
    __device__ static __forceinline__ M bld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return cvt(__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
    }
    __device__ static __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v) {
        __builtin_amdgcn_raw_buffer_store_b16(rne(v), r, vo, so, 0);
    }
    // Stochastic rounding for the values the time step accumulates into:
    // adding 16 uniform random bits below the kept ones and truncating
    // rounds up with probability equal to the dropped fraction, so
    // increments far below half an ulp still add up on average (with
    // round-to-nearest they vanish and slow flows stall).
    static constexpr bool kSR = true;
    __device__ static __forceinline__ void bst_r(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, M v,
                                                 uint32_t rbits) {
        const uint32_t u = __float_as_uint(v) + (rbits & 0xFFFFu);
        __builtin_amdgcn_raw_buffer_store_b16(uint16_t(u >> 16), r, vo, so, 0);
    }
};

// Counter-based 32-bit hash (the "lowbias32" xorshift-multiply mixer of
// C. Wellons' hash-prospector search): the random bits of stochastic
// rounding, a function of (step seed, node, population) only.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
template <class ST>
__device__ __forceinline__ uint32_t sr_bits(uint32_t hnode, int a) {
    if constexpr (ST::kSR) return mix32(hnode + uint32_t(a) * 0x85ebca77u);
    else return 0u;
}

// ---------------------------------------------------------- lane exchange
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane l <- lane l+1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane l <- lane l-1

template <int CTRL>
__device__ __forceinline__ float dpp(float src, float old) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double src, double old) {
    long long s = __double_as_longlong(src), o = __double_as_longlong(old);
    int slo = int(s & 0xffffffffll), shi = int(s >> 32);
    int olo = int(o & 0xffffffffll), ohi = int(o >> 32);
    int rlo = __builtin_amdgcn_update_dpp(olo, slo, CTRL, 0xf, 0xf, false);
    int rhi = __builtin_amdgcn_update_dpp(ohi, shi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)((unsigned long long)(unsigned)rlo |
                                            ((unsigned long long)(unsigned)rhi << 32)));
}

// Neighbour-lane value for the update kernel's x fluxes: a lane without a
// source lane (lane 0 for a right shift, 63 for a left shift) receives 0.
// Only the halo lanes 0, 1, 62 and 63 ever see such a value, or one
// derived from it, and their results are never stored; with no old value
// to merge, the shift is one instruction.
template <int CTRL>
__device__ __forceinline__ float nbr(float src) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double nbr(double src) {
    return dpp<CTRL>(src, src);
}

// The value of column col - 1 (xleft) or col + 1 (xright): the adjacent
// lane, or (WR: 8-column periodic lattice, eight columns per 8-lane group)
// the adjacent lane in the group with the wrap-around taken from the
// group's other end, by shifts inside the 16-lane DPP rows.
template <bool WR, class T>
__device__ __forceinline__ T xleft(T v, int col) {
    if constexpr (WR) {
        const T a = nbr<0x107>(v);   // row_shl:7, lane l <- l + 7
        const T b = nbr<0x111>(v);   // row_shr:1, lane l <- l - 1
        return col == 0 ? a : b;
    } else {
        return nbr<DPP_WAVE_SHR1>(v);
    }
}
template <bool WR, class T>
__device__ __forceinline__ T xright(T v, int col) {
    if constexpr (WR) {
        const T a = nbr<0x117>(v);   // row_shr:7, lane l <- l - 7
        const T b = nbr<0x101>(v);   // row_shl:1, lane l <- l + 1
        return col == 7 ? a : b;
    } else {
        return nbr<DPP_WAVE_SHL1>(v);
    }
}

// a wave-uniform value, made known as such to the compiler
__device__ __forceinline__ int64_t uniform(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t(uint64_t(lo) | (uint64_t(hi) << 32));
}
__device__ __forceinline__ void *uniform(char *p) {
    return reinterpret_cast<void *>(uniform(int64_t(reinterpret_cast<uintptr_t>(p))));
}

// minmod(a, b) = median(a, b, 0)
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b) {
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// ------------------------------------------------------------------ regions
__device__ __forceinline__ int reg_of(int lo, int hi, int j, const Geo &g) {
    if (j < lo || j > g.ny - hi) return REG_HIGH;
    if (g.iface == IF_PAPER && ((lo > 0 && j == lo) || (hi > 0 && j == g.ny - hi))) return REG_IFACE;
    return REG_LOW;
}
// the same rule with non-short-circuit operators: per-lane bands compile to
// selects instead of a divergent branch (a few more registers)
__device__ __forceinline__ int reg_of_sel(int lo, int hi, int j, const Geo &g) {
    const bool high = (j < lo) | (j > g.ny - hi);
    const bool ifc = (g.iface == IF_PAPER) & (((lo > 0) & (j == lo)) | ((hi > 0) & (j == g.ny - hi)));
    return high ? REG_HIGH : (ifc ? REG_IFACE : REG_LOW);
}
__device__ __forceinline__ int tile_of(int i, const Geo &g) { return g.ntiles == 1 ? 0 : i / g.tile_w; }
__device__ __forceinline__ int region_at(int i, int j, const Geo &g) {
    int t = tile_of(i, g);
    return reg_of(g.blo[t], g.bhi[t], j, g);
}

// Is a cross-neighbour within distance 2 of node (i, j) in region `want`?
// lo, hi: bands of the tile of column i.
__device__ bool neighbour_in(int i, int j, int want, int lo, int hi, const Geo &g) {
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        if (d == 0) continue;
        int jj = j + d;
        if (jj < 0 || jj > g.ny) {
            if (g.ybc != YBC_PERIODIC) continue;
            jj = (jj + g.nrow) % g.nrow;
        }
        if (reg_of(lo, hi, jj, g) == want) return true;
    }
    if (g.ntiles > 1) {
        int r = i % g.tile_w;
        if (r < 2 || r >= g.tile_w - 2) {
            int t = i / g.tile_w;
            for (int d = -2; d <= 2; ++d) {
                if (d == 0) continue;
                int ii = i + d;
                if (ii < 0 || ii >= g.nx) {
                    if (g.xbc != XBC_PERIODIC) continue;
                    ii = (ii + g.nx) % g.nx;
                }
                if (ii / g.tile_w != t && region_at(ii, j, g) == want) return true;
            }
        }
    }
    return false;
}

// ---------------------------------------------------- FP64 node arithmetic
template <class SS>
__device__ __forceinline__ double w_of(int a) {
    using TB = typename SS::T;
    return TB::rule.w[a % SS::N] * TB::rule.w[a / SS::N];
}

// rho, u of absolute populations (Eq. an, zeroth and first coefficients)
template <class SS>
__device__ void moments_d(const double *f, double &rho, double &ux, double &uy) {
    using TB = typename SS::T;
    double r = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) {
        r += f[a];
        jx += TB::rule.x[a % SS::N] * f[a];
        jy += TB::rule.x[a / SS::N] * f[a];
    }
    rho = r;
    ux = jx / r;
    uy = jy / r;
}

// Hermite coefficients of the 1D Maxwellian factor at velocity u and
// temperature 1 + th, h_0 .. h_{K-1}: h_0 = 1, h_1 = u,
// h_{k+1} = u h_k + k th h_{k-1} (the three-term recurrence of He_k carried
// over to the Gaussian's moments); isothermal sets (TH false) take
// th = 0, h_k = u^k.
template <bool TH, int K, class T>
__device__ __forceinline__ void hcoef(T u, T th, T (&h)[K]) {
    h[0] = T(1);
#pragma unroll
    for (int k = 1; k < K; ++k) {
        if constexpr (TH) h[k] = k >= 2 ? u * h[k - 1] + T(k - 1) * th * h[k - 2] : h[k - 1] * u;
        else h[k] = h[k - 1] * u;
    }
}

// rho, u and th = T - 1 of absolute populations: T from the energy moment,
// sum xi^2 f = rho (u^2 + 2 T), on thermal sets; th = 0 otherwise
template <class SS>
__device__ void moments_td(const double *f, double &rho, double &ux, double &uy, double &th) {
    moments_d<SS>(f, rho, ux, uy);
    th = 0.0;
    if constexpr (SS::TH) {
        using TB = typename SS::T;
        double e = 0.0;
#pragma unroll
        for (int a = 0; a < SS::Q; ++a) {
            const double x = TB::rule.x[a % SS::N], y = TB::rule.x[a / SS::N];
            e += (x * x + y * y) * f[a];
        }
        th = 0.5 * (e / rho - (ux * ux + uy * uy)) - 1.0;
    }
}

// Order-EQ Hermite equilibrium (Eq. approxfeq) at temperature 1 + th (th
// ignored unless SS is thermal), absolute values
template <class SS>
__device__ void feq_d(double rho, double ux, double uy, double th, double *out) {
    using TB = typename SS::T;
    constexpr int N = SS::N, EQ = SS::EQ;
    double px[EQ + 1], py[EQ + 1];
    hcoef<SS::TH>(ux, th, px);
    hcoef<SS::TH>(uy, th, py);
#pragma unroll
    for (int q = 0; q < N; ++q) {
        double B[EQ + 1];
#pragma unroll
        for (int k = 0; k <= EQ; ++k) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m + k <= EQ; ++m) s += py[m] * TB::hk.v[m][q];
            B[k] = s * px[k];
        }
#pragma unroll
        for (int p = 0; p < N; ++p) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k <= EQ; ++k) s += TB::hk.v[k][p] * B[k];
            out[p + N * q] = TB::rule.w[p] * TB::rule.w[q] * rho * s;
        }
    }
}

// Hermite-moment projection from set SS to set DD (FP64):
// equilibrium rebuilt in DD from rho, u; non-equilibrium coefficients a_km -
// a_eq,km carried for k, m below both sets' point counts; the rest from the
// closure (NULL = 0).  A set projected on itself is copied.
template <class SS, class DD>
__device__ void project_d(const double *fs, double *fd, const double *closure) {
    if constexpr (SS::N == DD::N && SS::EQ == DD::EQ) {
#pragma unroll
        for (int a = 0; a < SS::Q; ++a) fd[a] = fs[a];
    } else {
        using TS = typename SS::T;
        using TD = typename DD::T;
        constexpr int NS = SS::N, ND = DD::N;
        constexpr int NM = NS < ND ? NS : ND;
        double t[NS][NM];
#pragma unroll
        for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < NS; ++q) s += fs[p + NS * q] * TS::he.v[m][q];
                t[p][m] = s;
            }
        double a[NM][NM];
#pragma unroll
        for (int k = 0; k < NM; ++k)
#pragma unroll
            for (int m = 0; m < NM; ++m) {
                double s = 0.0;
#pragma unroll
                for (int p = 0; p < NS; ++p) s += TS::he.v[k][p] * t[p][m];
                a[k][m] = s;
            }
        const double rho = a[0][0], ux = a[1][0] / rho, uy = a[0][1] / rho;
        // thermal: the node's temperature from a_20 + a_02 = rho (u^2 + 2 (T - 1))
        const double th = SS::TH ? 0.5 * ((a[2][0] + a[0][2]) / rho - (ux * ux + uy * uy)) : 0.0;
        double px[ND + 1], py[ND + 1];
        hcoef<SS::TH>(ux, th, px);
        hcoef<SS::TH>(uy, th, py);
        double c[ND][ND];
#pragma unroll
        for (int k = 0; k < ND; ++k)
#pragma unroll
            for (int m = 0; m < ND; ++m) {
                double eqd = (k + m <= DD::EQ) ? rho * px[k] * py[m] : 0.0;
                double neq;
                if (k < NM && m < NM) {
                    double eqs = (k + m <= SS::EQ) ? rho * px[k] * py[m] : 0.0;
                    neq = a[k][m] - eqs;
                } else {
                    neq = closure ? closure[k * ND + m] : 0.0;
                }
                c[k][m] = eqd + neq;
            }
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            double B[ND];
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                double s = 0.0;
#pragma unroll
                for (int m = 0; m < ND; ++m) s += c[k][m] * TD::hk.v[m][q];
                B[k] = s;
            }
#pragma unroll
            for (int p = 0; p < ND; ++p) {
                double s = 0.0;
#pragma unroll
                for (int k = 0; k < ND; ++k) s += TD::hk.v[k][p] * B[k];
                fd[p + ND * q] = TD::rule.w[p] * TD::rule.w[q] * s;
            }
        }
    }
}

// ---------------------------------------------------- node stores (FP64 in)
template <class ST, class SS>
__device__ __forceinline__ typename ST::S *plane0(const Buf &b, int copy) {
    return reinterpret_cast<typename ST::S *>(b.base[copy]) + b.rowbase;
}

// storage reference of column i (Shift): s0 + ds * floor(i / SHIFT_GROUP)
__device__ __forceinline__ int shift_group(int i) {
    return i >= 0 ? i / SHIFT_GROUP : (i - (SHIFT_GROUP - 1)) / SHIFT_GROUP;
}
__device__ __forceinline__ double shift_at(const Shift &s, int i) { return s.s0 + s.ds * double(shift_group(i)); }

template <class A>
__device__ __forceinline__ Shift sh_of(const A &a) { return Shift{a.rho_shift, a.dshift}; }

template <class ST, class SS>
__device__ void load_node_d(const Buf &b, int copy, int i, int j, const Shift &sh, double *f) {
    const typename ST::S *p = plane0<ST, SS>(b, copy) + (int64_t)(j + 2) * b.pitch + i;
    const double shift = shift_at(sh, i);
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) f[a] = ST::ldd(p + a * b.plane) + w_of<SS>(a) * shift;
}

// absolute populations f to node / ghost entry (i, j), shifted by the
// reference of column i
template <class ST, class SS>
__device__ void store_node_d(const Buf &b, int copy, int i, int j, const Shift &sh, const double *f) {
    typename ST::S *p = plane0<ST, SS>(b, copy) + (int64_t)(j + 2) * b.pitch + i;
    const double shift = shift_at(sh, i);
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) ST::std_(p + a * b.plane, f[a] - w_of<SS>(a) * shift);
}

// Write node (i, j)'s populations f (set SS, absolute) to (i, j) when
// `own`, and to every ghost entry that stands for it: the wall ghost rows
// (Sec. 3.2: copies of the wall node), periodic images, and the pressure
// boundary columns (equilibrium at the prescribed density with the edge
// node's velocity and temperature plus the edge node's non-equilibrium
// part).
template <class ST, class SS>
__device__ void emit_node(const Buf &b, int copy, int i, int j, const Shift &shift, const double *f, bool own,
                          const Geo &g, const Phys &ph) {
    if (own) store_node_d<ST, SS>(b, copy, i, j, shift, f);
    if (g.ybc == YBC_WALLS) {
        if (j == 0) {
            store_node_d<ST, SS>(b, copy, i, -1, shift, f);
            store_node_d<ST, SS>(b, copy, i, -2, shift, f);
        }
        if (j == g.ny) {
            store_node_d<ST, SS>(b, copy, i, g.ny + 1, shift, f);
            store_node_d<ST, SS>(b, copy, i, g.ny + 2, shift, f);
        }
    } else if (g.ybc == YBC_SHEAR) {
        if (j == 0) {
            store_node_d<ST, SS>(b, copy, i, -1, shift, f);
            store_node_d<ST, SS>(b, copy, i, -2, shift, f);
        }
        if (j == g.ny) {
            // imposed shear (Kramers' problem, Sec. 3.3): equilibrium at the
            // node's density (and temperature) with its velocity raised by
            // shear * k, plus the node's non-equilibrium part
            double rho, ux, uy, th, en[SS::Q], eg[SS::Q], gq[SS::Q];
            moments_td<SS>(f, rho, ux, uy, th);
            feq_d<SS>(rho, ux, uy, th, en);
            for (int k = 1; k <= 2; ++k) {
                feq_d<SS>(rho, ux + ph.shear * double(k), uy, th, eg);
#pragma unroll
                for (int a = 0; a < SS::Q; ++a) gq[a] = eg[a] + (f[a] - en[a]);
                store_node_d<ST, SS>(b, copy, i, g.ny + k, shift, gq);
            }
        }
    } else {
        if (j < 2) store_node_d<ST, SS>(b, copy, i, j + g.nrow, shift, f);
        if (j >= g.nrow - 2) store_node_d<ST, SS>(b, copy, i, j - g.nrow, shift, f);
    }
    if (g.xbc == XBC_PERIODIC) {
        if (i < 2) store_node_d<ST, SS>(b, copy, i + g.nx, j, shift, f);
        if (i >= g.nx - 2) store_node_d<ST, SS>(b, copy, i - g.nx, j, shift, f);
    } else if (i == 0 || i == g.nx - 1) {
        double rho, ux, uy, th, eb[SS::Q], en[SS::Q], gq[SS::Q];
        moments_td<SS>(f, rho, ux, uy, th);
        feq_d<SS>(i == 0 ? ph.rho_in : ph.rho_out, ux, uy, th, eb);
        feq_d<SS>(rho, ux, uy, th, en);
#pragma unroll
        for (int a = 0; a < SS::Q; ++a) gq[a] = eb[a] + (f[a] - en[a]);
        if (i == 0) {
            store_node_d<ST, SS>(b, copy, -1, j, shift, gq);
            store_node_d<ST, SS>(b, copy, -2, j, shift, gq);
        } else {
            store_node_d<ST, SS>(b, copy, g.nx, j, shift, gq);
            store_node_d<ST, SS>(b, copy, g.nx + 1, j, shift, gq);
        }
    }
}

// Everything a node of set SS owes the next step besides its own entry:
// images, and (Hermite interface) its projection into the partner set OO
// wherever a stencil of OO reads it.
template <class ST, class SS, class OO>
__device__ void finish_node(const Buf &self, const Buf &other, int copy, int i, int j, const Shift &shift,
                            const double *f, bool own, bool proj, const Geo &g, const Phys &ph) {
    emit_node<ST, SS>(self, copy, i, j, shift, f, own, g, ph);
    if constexpr (OO::Q > 0) {
        if (proj) {
            double fo[OO::Q];
            project_d<SS, OO>(f, fo, nullptr);
            emit_node<ST, OO>(other, copy, i, j, shift, fo, true, g, ph);
        }
    }
}

// ------------------------------------------------------------- hot kernel
// One time step of set SS.  A work item is a group of 60 columns
// [i0, i0+60) x a strip of rows [j0, j1).  The block has SPLIT waves; every
// wave holds the same 64 columns [i0-2, i0+62) (the two extra columns on each
// side are halo lanes that load but never store) and evolves the
// populations of N/SPLIT of the set's y-abscissae, so per row a wave issues
// one load and one store per population it owns -- well inside the 63
// outstanding vector-memory operations a wave can track -- and needs about a
// hundred registers.  The partial moments are exchanged through LDS (one
// barrier per row) and summed in a fixed order, so every wave of the block
// sees bit-identical rho and u.
//
// Loads are software-pipelined: as soon as a population's value for the
// current row has been consumed, the load of its next-row value is issued,
// so a whole row of arithmetic covers the memory latency.  Each lane marches
// up its column keeping, per population, the values and limited slopes the
// y fluxes need; x neighbours come from neighbouring lanes by DPP wave
// shifts.
//
// Diffuse walls (Sec. 3.2) are applied on wall rows inside the kernel (a
// wall row is the same for the whole block): the flux into the wall,
// n = sum |xi_y| f over the populations moving into the wall, is reduced over
// the block; the populations leaving the wall are then rho_W S(u_wall) with
// rho_W = n / sum_leaving |xi_y| S.  With the storage shift s (stored
// f' = f - w s) and S = w + S', this becomes f' = d w + (d + s) S' with
// d = (n' - s D') / (K + D'), K = sum_leaving |xi_y| w,
// D' = sum_leaving |xi_y| S' and n' the flux of the stored values, so no
// large quantities cancel in FP32.
template <class SS>
constexpr int update_split() { return SS::Q == 36 ? LB_SPLIT36 : SS::Q == 16 ? 2 : 1; }
// the same for the high set of the merged launch with D2Q9 (k_update_pair)
template <class SS>
constexpr int pair_split() { return SS::Q == 36 ? LB_PAIR_SPLIT36 : update_split<SS>(); }
// ... and in the batch update
template <class SS>
constexpr int multi_split() { return SS::Q == 36 ? LB_MULTI_SPLIT36 : SS::Q == 16 ? LB_MULTI_SPLIT16 : 1; }

// LDS of a split update: per y-abscissa partial moments (double-buffered
// by row) and wall fluxes; one allocation per set and split
template <class T, int N, int SPLIT>
__device__ __forceinline__ T (*lds_moments())[2][N][64] {
    __shared__ T sm[2][2][N][64];
    return sm;
}
template <class T, int N, int SPLIT>
__device__ __forceinline__ T (*lds_wall())[N][64] {
    __shared__ T sn[2][N][64];
    return sn;
}
// ... and, on thermal sets, the per y-abscissa energy sums (double-buffered)
template <class T, int N, int SPLIT>
__device__ __forceinline__ T (*lds_energy())[N][64] {
    __shared__ T se[2][N][64];
    return se;
}

// occupancy the compiler must fit the update kernel into (waves per SIMD)
template <class SS>
constexpr int update_waves() { return SS::Q == 36 ? LB_WAVES36 : SS::Q == 16 ? 4 : 6; }
// the same for the merged and batched update kernels (more code paths)
template <class SS>
constexpr int pair_waves() { return SS::Q == 36 ? LB_WAVES36_PAIR : update_waves<SS>(); }

// load of a stored population, moved by w * dl to another storage
// reference when XS (FP32 arithmetic, fused within the expression)
template <class ST, bool XS>
__device__ __forceinline__ typename ST::M ld_x(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so,
                                               typename ST::M w, typename ST::M dl) {
#pragma clang fp contract(on)
    typename ST::M v = ST::bld(r, vo, so);
    if constexpr (XS) v = v + w * dl;
    return v;
}

template <class ST, class SS, class OO, int WV, bool NW = false, int SPL = update_split<SS>(), bool WR = false,
          bool XS = false>
__device__ __forceinline__ void update_rows(const StepArgs &A, const int cur, const uint32_t seed, const int i0,
                                            const int j0, const int j1, const int lane, const int S = 0);

// one work item of one lattice: 64 columns x rows j0..j1, or (NW, a
// narrow lattice) 64 / (nx + 4) lane groups of nx + 4 columns each, group
// g marching rows j0 + g S .. j0 + (g + 1) S (clipped to j1); SPL waves
// share the populations (the result does not depend on SPL)
template <class ST, class SS, class OO, bool NW = false, int SPL = update_split<SS>(), bool WR = false,
          bool XS = false>
__device__ __forceinline__ void update_item(const StepArgs &A, const int cur, const uint32_t seed, const int i0,
                                            const int j0, const int j1, const int S = 0) {
    constexpr int SPLIT = SPL;
    const int lane = threadIdx.x & 63;
    // the wave index is wave-uniform: each wave runs the row loop compiled
    // for its own abscissae, so every population's upwind direction and
    // constants are known at compile time
    const int wv = SPLIT > 1 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6) : 0;
    if (wv == 0) update_rows<ST, SS, OO, 0, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
    if constexpr (SPLIT > 1) {
        if (wv == 1) update_rows<ST, SS, OO, 1, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
    }
    if constexpr (SPLIT > 2) {
        if (wv == 2) update_rows<ST, SS, OO, 2, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
    }
    if constexpr (SPLIT > 3) {
        if (wv == 3) update_rows<ST, SS, OO, 3, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
        if (wv == 4) update_rows<ST, SS, OO, 4, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
        if (wv == 5) update_rows<ST, SS, OO, 5, NW, SPL, WR, XS>(A, cur, seed, i0, j0, j1, lane, S);
    }
}

// XS: the storage reference varies by column group (FP32 / BF16 pressure
// lattices): the variant that moves other groups' loaded values to the
// item's reference (a kernel of its own, so the common one is unchanged)
template <class ST, class SS, class OO, bool XS = false>
__global__ __launch_bounds__(64 * update_split<SS>())
__attribute__((amdgpu_waves_per_eu(sizeof(typename ST::M) == 8 ? 2 : update_waves<SS>())))
void k_update(const StepArgs A) {
    // XCD-aware mapping: consecutive items (neighbouring strips) go to
    // blocks that the dispatcher places on the same XCD (block b -> XCD b % 8)
    const int b = blockIdx.x;
    const int it = (b & 7) * A.chunk + (b >> 3);
    if (it >= A.nitems) return;
    const int i0 = A.items[4 * it], j0 = A.items[4 * it + 1], j1 = A.items[4 * it + 2];
    if (j0 >= j1) return;   // padding item
    update_item<ST, SS, OO, false, update_split<SS>(), false, XS>(A, A.cur, A.seed, i0, j0, j1);
}

// Both sets of a lattice in one launch, for a D2Q9 low set (one wave per
// item): the first nb_h blocks run the high set's items (SPLIT waves per
// item, as k_update), the rest give each of their SPLIT waves its own
// D2Q9 item.  The two sets touch disjoint buffers, and one launch lets
// their waves share the machine instead of running back to back.

template <class ST, class LS, class HS, bool XS = false>
__global__ __launch_bounds__(64 * pair_split<HS>())
__attribute__((amdgpu_waves_per_eu(sizeof(typename ST::M) == 8 ? 2 : pair_waves<HS>())))
void k_update_pair(const StepArgs L, const StepArgs H, const int nb_h) {
    if constexpr (update_split<LS>() == 1) {
        constexpr int SPLIT = pair_split<HS>();
        const int b = blockIdx.x;
        if (b < nb_h) {
            const int it = (b & 7) * H.chunk + (b >> 3);
            if (it >= H.nitems) return;
            const int i0 = H.items[4 * it], j0 = H.items[4 * it + 1], j1 = H.items[4 * it + 2];
            if (j0 >= j1) return;
            update_item<ST, HS, LS, false, SPLIT, false, XS>(H, H.cur, H.seed, i0, j0, j1);
        } else {
            // low items: XCD slab (b' mod 8) of L.chunk items, SPLIT per block
            const int bl = b - nb_h;
            const int w = SPLIT > 1 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6) : 0;
            const int pos = SPLIT * (bl >> 3) + w;
            if (pos >= L.chunk) return;
            const int it = (bl & 7) * L.chunk + pos;
            if (it >= L.nitems) return;
            const int i0 = L.items[4 * it], j0 = L.items[4 * it + 1], j1 = L.items[4 * it + 2];
            if (j0 >= j1) return;
            update_rows<ST, LS, HS, 0, false, update_split<LS>(), false, XS>(L, L.cur, L.seed, i0, j0, j1,
                                                                          threadIdx.x & 63);
        }
    }
}

// The update of a batch of independent lattices, every velocity set in one
// launch.  Item (i0, j0, j1, l) belongs to lattice (and side) l, whose
// arguments are M.desc[l]; the lattices of a batch step together, so the
// copy parity is the launch's.  Blocks have multi_waves() waves: a D2Q36
// or D2Q16 item takes as many as its split (waves left over leave at once:
// a barrier waits only for the waves still running), and a D2Q9 item a
// single wave, multi_waves() to a block (S36 and S16 are the D2Q36 and D2Q16 sets of the
// batch, of their equilibrium orders).  Within each slot the blocks are
// mapped to items XCD by XCD as in the single-lattice kernels (slot starts
// are multiples of 8).
template <class ST, class SS>
__device__ __forceinline__ void batch_item(const BatchMulti &M, const int slot, const int it) {
    if (it >= M.nitems[slot]) return;
    const int32_t *e = M.items[slot] + 4 * it;
    const int i0 = __builtin_amdgcn_readfirstlane(e[0]);
    const int j0 = __builtin_amdgcn_readfirstlane(e[1]);
    const int j1 = __builtin_amdgcn_readfirstlane(e[2]);
    const int l = __builtin_amdgcn_readfirstlane(e[3]);
    if (j0 >= j1) return;   // padding item
    // the table is read through the constant address space: the lattice's
    // arguments are then scalar loads, as they are for a single lattice
    // (through a generic pointer the compiler cannot rule out that the
    // kernel's own stores change them, and reloads them per lane)
    const StepArgs &A = *(const StepArgs *)((const __attribute__((address_space(4))) StepArgs *)M.desc + l);
    // a negative first column marks a narrow lattice's item: -i0 rows per
    // lane group, or -i0 - NW_WRAP for an 8-column periodic lattice whose
    // x neighbours wrap inside 8-lane groups
    if (i0 <= -NW_WRAP) {
        update_item<ST, SS, SS, true, multi_split<SS>(), true>(A, M.cur, M.seed, 0, j0, j1, -i0 - NW_WRAP);
        return;
    }
    if constexpr (sizeof(typename ST::M) == 4) {
        if (A.dshift != 0.0) {
            if (i0 < 0) update_item<ST, SS, SS, true, multi_split<SS>(), false, true>(A, M.cur, M.seed, 0, j0, j1, -i0);
            else update_item<ST, SS, SS, false, multi_split<SS>(), false, true>(A, M.cur, M.seed, i0, j0, j1);
            return;
        }
    }
    if (i0 < 0) update_item<ST, SS, SS, true, multi_split<SS>()>(A, M.cur, M.seed, 0, j0, j1, -i0);
    else update_item<ST, SS, SS, false, multi_split<SS>()>(A, M.cur, M.seed, i0, j0, j1);
}

// waves per block of the batch update: enough for a D2Q36 or a D2Q16 item
constexpr int multi_waves() { return LB_MULTI_SPLIT36 > LB_MULTI_SPLIT16 ? LB_MULTI_SPLIT36 : LB_MULTI_SPLIT16; }

template <class ST, class S36, class S16>
__global__ __launch_bounds__(64 * multi_waves())
__attribute__((amdgpu_waves_per_eu(sizeof(typename ST::M) == 8 ? 2 : LB_MULTI_WAVES)))
void k_update_multi(const BatchMulti M) {
    using S9 = lbt::VSet<3, 2>;
    constexpr int MW = multi_waves();
    static_assert(multi_split<S36>() <= MW && multi_split<S16>() <= MW && multi_split<S9>() == 1,
                  "an item's waves fit a block");
    const int b = blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    if (b < M.start[1]) {
        if (w < multi_split<S36>()) batch_item<ST, S36>(M, 0, (b & 7) * M.nsplit[0] + (b >> 3));
    } else if (b < M.start[2]) {
        const int bl = b - M.start[1];
        if (w < multi_split<S16>()) batch_item<ST, S16>(M, 1, (bl & 7) * M.nsplit[1] + (bl >> 3));
    } else {
        const int bl = b - M.start[2];
        const int pos = MW * (bl >> 3) + w;
        if (pos < M.nsplit[2]) batch_item<ST, S9>(M, 2, (bl & 7) * M.nsplit[2] + pos);
    }
}

// store of an updated value of population a in row j: stochastically
// rounded where the storage type does that (bf16), plain otherwise.  The
// random bits hash the step seed, the row and the population but not the
// column: every copy of a value rounds alike, and a state uniform in x
// stays uniform in x (the unsplit update is stable at Courant 0.5 only for
// such states; column-dependent noise would seed growing 2D modes).
#define LB_ST(voff, soff, val)                                                           \
    {                                                                                    \
        if constexpr (ST::kSR) {                                                         \
            ST::bst_r(rd, voff, soff, val, sr_bits<ST>(uint32_t(j) * 0x9e3779b1u ^ seed, a)); \
        } else {                                                                         \
            ST::bst(rd, voff, soff, val);                                                \
        }                                                                                \
    }

template <class ST, class SS, class OO, int WV, bool NW, int SPL, bool WR, bool XS>
__device__ __forceinline__ void update_rows(const StepArgs &A, const int cur, const uint32_t seed, const int i0,
                                            const int j0, const int j1, const int lane, const int S) {
    // multiply-adds are fused within an expression only (not across
    // statements, where the choice would depend on the surrounding code):
    // every instantiation (split, narrow or wide, merged or alone) then
    // rounds a population's update the same way
#pragma clang fp contract(on)
    using T = typename ST::M;
    using SV = typename ST::S;
    using TB = typename SS::T;
    constexpr int N = SS::N, Q = SS::Q, EQ = SS::EQ;
    constexpr int SPLIT = SPL;
    constexpr int NQ = N / SPLIT;      // y-abscissae per wave
    constexpr int QW = NQ * N;         // populations per wave
    constexpr int q0 = WV * NQ;
    constexpr int wv = WV;
    static_assert(N % SPLIT == 0, "split must divide the abscissae");
    // a copy, read once up front: a batch's lattice arguments come from a
    // device table, and a field first read under a per-lane condition
    // (e.g. ny in the ownership test) would otherwise be reloaded there and
    // merged into a per-lane register
    const Geo g = A.g;
    const int nx = g.nx;
    // narrow lattices: lane group gl of nx + 4 lanes (2 halo columns each
    // side) marches its own rows [jl0, jl1); wide: one group, rows [j0, j1)
    int col, jl0 = j0, jl1 = j1;
    bool valid;
    if constexpr (WR) {
        // 8-column periodic lattices: eight groups of eight lanes, the x
        // neighbours wrapped inside the group (no halo lanes)
        const int gl = lane >> 3;
        col = lane & 7;
        jl0 = min(j0 + gl * S, j1);
        jl1 = min(jl0 + S, j1);
        valid = true;
    } else if constexpr (NW) {
        const int G = nx + 4, gl = lane / G;
        col = lane - gl * G - 2;
        jl0 = min(j0 + gl * S, j1);
        jl1 = min(jl0 + S, j1);
        valid = gl < 64 / G && col >= 0 && col < nx;
    } else {
        col = i0 - 2 + lane;
        valid = lane >= 2 && lane < 62 && col < nx;
    }

    // Addressing: raw buffer access with one descriptor per copy, the lane's
    // 32-bit byte offset (counted from column -2) in a vector register and
    // the wave-uniform offset of (population, row) in a scalar register.
    // Lanes that must not store get an offset past the end of the buffer,
    // which the hardware turns into a dropped store (or a zero load).
    // Why this does not depend on how the compiler distributes an address
    // over the vector, scalar and immediate offset fields: the host refuses
    // lattices whose population buffer per set and copy reaches 2^31 bytes,
    // so nbytes, every in-range byte offset and every scalar offset are
    // below 2^31.  An in-range access has a total offset below nbytes
    // whatever part of it sits in which field; a masked access has a vector
    // part of at least nbytes (OOB, plus a non-negative row offset below
    // 2^31 for narrow lattices), so vector + immediate (+ scalar, where the
    // check counts it) stays in [nbytes, 2^32): it cannot wrap into range.
    // Moving a uniform term between fields only adds a non-negative amount
    // below 2^31 to the vector part; per-lane selects cannot move to the
    // scalar field.
    // (the lattice's arguments are wave-uniform; a batch reads them from a
    // device table, so they are declared uniform here: the descriptor and
    // the scalar offsets must live in scalar registers)
    constexpr unsigned EB = sizeof(SV);
    const int64_t P = uniform(A.self.plane);
    const int64_t pitch = uniform(int64_t(A.self.pitch));
    const int64_t rb = uniform(int64_t(A.self.rowbase - 2));
    const unsigned nbytes = unsigned(int64_t(Q) * P * EB);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(uniform(A.self.base[cur]), 0, int(nbytes), 0x00020000);
    const __amdgpu_buffer_rsrc_t rd =
        __builtin_amdgcn_make_buffer_rsrc(uniform(A.self.base[cur ^ 1]), 0, int(nbytes), 0x00020000);
    const unsigned OOB = nbytes;
    const unsigned vl = unsigned(min(max(col, -2), nx + 1) + 2) * EB;
    // storage reference of this item: every node it owns lies in one column
    // group (a wide item's 60 columns start at a multiple of 60, a narrow
    // lattice has fewer than 60 columns).  XS: values of lanes in another
    // group (halo lanes, ghost columns) are moved to this item's reference
    // as they are loaded, + w_alpha (s(column) - s(item))
    const Shift shv = sh_of(A);
    const double s_item = XS ? shift_at(shv, NW ? 0 : i0) : A.rho_shift;
    T dl = T(0);
    if constexpr (XS) dl = T(shift_at(shv, min(max(col, -2), nx + 1)) - s_item);
#define LB_LD(a, vo, so) \
    ld_x<ST, XS>(rs, vo, so, T(TB::rule.w[(a) % N] * TB::rule.w[(a) / N]), dl)
#define LB_SOFF(a, j) unsigned(((int64_t)(a) * P + rb + (int64_t)((j) + 2) * pitch) * EB)
    // narrow lattices: the row is per lane, so it moves into the vector
    // offset and the scalar offset keeps the population only
#define LB_VO(v, j) ((NW || LB_ROWV) ? (v) + unsigned((int64_t)((j) + 2) * pitch * EB) : (v))
#define LB_SO(a, j) ((NW || LB_ROWV) ? unsigned(((int64_t)(a) * P + rb) * EB) : LB_SOFF(a, j))

    // region ownership of this lane's column (bands of its tile)
    const int tl = tile_of(min(max(col, 0), nx - 1), g);
    const int lo_l = g.blo[tl], hi_l = g.bhi[tl];
    const int want = A.self_high ? REG_HIGH : REG_LOW;

    // per-abscissa constants nu_p = x_p dt and k_p = |nu_p|(1 - |nu_p|)/2
    T nu[N], kk[N];
#pragma unroll
    for (int p = 0; p < N; ++p) {
        if constexpr (sizeof(T) == 8) {
            nu[p] = A.ks.nu[p];
            kk[p] = A.ks.kk[p];
        } else {
            nu[p] = A.ks.nuf[p];
            kk[p] = A.ks.kkf[p];
        }
    }

    // wave-local population index a = p + N * (q0 + qq), qq < NQ
#define LB_POP(k) ((k) % N + N * (q0 + (k) / N))
    // first row's next-row values, issued together with the window
    T nw[QW];
#pragma unroll
    for (int k = 0; k < QW; ++k) {
        const double xq = TB::rule.x[q0 + k / N];
        nw[k] = LB_LD(LB_POP(k), LB_VO(vl, xq < 0.0 ? jl0 + 2 : jl0 + 1),
                      LB_SO(LB_POP(k), xq < 0.0 ? jl0 + 2 : jl0 + 1));
    }
    // y window per population: c = f_j; for xi_y > 0: s1 = f_j - f_{j-1},
    // s2 = minmod(f_{j-1} - f_{j-2}, f_j - f_{j-1}); for xi_y < 0:
    // s1 = f_{j+1}, s2 = minmod(f_{j+1} - f_j, f_j - f_{j-1})
    T c[QW], s1[QW], s2[QW];
#pragma unroll
    for (int k = 0; k < QW; ++k) {
        const int a = LB_POP(k);
        const double xq = TB::rule.x[q0 + k / N];
        if (xq > 0.0) {
            T fm2 = LB_LD(a, LB_VO(vl, jl0 - 2), LB_SO(a, jl0 - 2));
            T fm1 = LB_LD(a, LB_VO(vl, jl0 - 1), LB_SO(a, jl0 - 1));
            T f0 = LB_LD(a, LB_VO(vl, jl0), LB_SO(a, jl0));
            c[k] = f0;
            s1[k] = f0 - fm1;
            s2[k] = minmod(fm1 - fm2, f0 - fm1);
        } else if (xq < 0.0) {
            T fm1 = LB_LD(a, LB_VO(vl, jl0 - 1), LB_SO(a, jl0 - 1));
            T f0 = LB_LD(a, LB_VO(vl, jl0), LB_SO(a, jl0));
            T fp1 = LB_LD(a, LB_VO(vl, jl0 + 1), LB_SO(a, jl0 + 1));
            c[k] = f0;
            s1[k] = fp1;
            s2[k] = minmod(fp1 - f0, f0 - fm1);
        } else {
            c[k] = LB_LD(a, LB_VO(vl, jl0), LB_SO(a, jl0));
            s1[k] = T(0);
            s2[k] = T(0);
        }
    }

    // periodic images of the first/last two columns are written here; row
    // images, pressure columns and partner-set projections are finished
    // afterwards by k_finish / k_project_halo
    const bool per_x = g.xbc == XBC_PERIODIC;
    const bool wave_img = per_x && (NW || i0 < 2 || i0 + 60 > nx - 2);   // uniform

    const T rho_shift = T(s_item);
    const T om0 = T(A.ph.omega0);
    const T om_rho = T(A.ph.omega0 / A.ph.rho_ref);
    const T dtT = T(A.ph.dt), gxT = T(A.ph.gx), gyT = T(A.ph.gy);

    // LDS: per-abscissa partial moments (double-buffered by row) and wall
    // fluxes, shared by the wave variants
    T (*sm)[2][N][64] = lds_moments<T, N, SPLIT>();
    T (*sn)[N][64] = lds_wall<T, N, SPLIT>();

    // (narrow: the loop counts a group's rows, S for every group)
    for (int jr = NW ? 0 : j0; jr < (NW ? S : j1); ++jr) {
        const int j = NW ? jl0 + jr : jr;
        const bool more = jr + 1 < (NW ? S : j1);
        const unsigned vln = more ? vl : OOB;
        // (without short-circuit: selects, not a divergent branch, for the
        // sets whose register budget leaves room; D2Q36 would spill)
        const int rj = Q < 36 ? reg_of_sel(lo_l, hi_l, j, g) : reg_of(lo_l, hi_l, j, g);
        const bool own = valid & (!NW || j < jl1) & (rj == want);
        const unsigned vs = own ? unsigned(col + 2) * EB : OOB;
        const unsigned vimg_lo = (per_x && own && col < 2) ? unsigned(col + nx + 2) * EB : OOB;
        const unsigned vimg_hi = (per_x && own && col >= nx - 2) ? unsigned(col - nx + 2) * EB : OOB;
        // wall rows: uniform for a wide item; per lane group for a narrow
        // one, whose wall code runs when any lane has a wall row and only
        // stores from those lanes
        const bool wall_l = (j == 0 ? g.ybc != YBC_PERIODIC : (j == g.ny && g.ybc == YBC_WALLS)) && (!NW || j < jl1);
        const bool wall = NW ? __builtin_amdgcn_ballot_w64(wall_l) != 0 : wall_l;
        const unsigned vw = NW ? (wall_l ? vs : OOB) : vs;
        const bool bottom = j == 0;
        const int gj1 = bottom ? -1 : g.ny + 1, gj2 = bottom ? -2 : g.ny + 2;
        // flux of the stored values into the wall: per y-abscissa partial
        // sums (nq), summed over the abscissae in order like the moments
        T nacc = T(0);

        // moments of the centre values: rho' = sum f (shifted), j = sum xi f
        // (thermal sets: also e' = sum |xi|^2 f, shifted).  Per y-abscissa
        // partial sums, then summed over the abscissae in order (through LDS
        // when the populations are split over waves), so the moments do not
        // depend on the split.
        T sqv[NQ], sxv[NQ], sev[NQ];
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            T sq = T(0), sxq = T(0), seq = T(0);
#pragma unroll
            for (int p = 0; p < N; ++p) {
                sq += c[p + N * qq];
                sxq += T(TB::rule.x[p]) * c[p + N * qq];
                if constexpr (SS::TH) seq += T(TB::rule.x[p] * TB::rule.x[p]) * c[p + N * qq];
            }
            sqv[qq] = sq;
            sxv[qq] = sxq;
            sev[qq] = seq;
        }
        T rp = T(0), jx = T(0), jy = T(0), ep = T(0);
        if constexpr (SPLIT == 1) {
#pragma unroll
            for (int q = 0; q < N; ++q) {
                rp += sqv[q];
                jx += sxv[q];
                jy += T(TB::rule.x[q]) * sqv[q];
                if constexpr (SS::TH) ep += sev[q] + T(TB::rule.x[q] * TB::rule.x[q]) * sqv[q];
            }
        } else {
            const int buf = NW ? jr & 1 : (j - j0) & 1;
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq) {
                sm[buf][0][q0 + qq][lane] = sqv[qq];
                sm[buf][1][q0 + qq][lane] = sxv[qq];
                if constexpr (SS::TH) lds_energy<T, N, SPLIT>()[buf][q0 + qq][lane] = sev[qq];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const T sq = sm[buf][0][q][lane];
                rp += sq;
                jx += sm[buf][1][q][lane];
                jy += T(TB::rule.x[q]) * sq;
                if constexpr (SS::TH)
                    ep += lds_energy<T, N, SPLIT>()[buf][q][lane] + T(TB::rule.x[q] * TB::rule.x[q]) * sq;
            }
        }
        const T rho = rho_shift + rp;
        const T inv = T(1) / rho;
        const T ux = jx * inv, uy = jy * inv;
        // thermal: T - 1 from sum |xi|^2 f - 2 rho = e' - 2 rho' (the shift
        // s carries sum w |xi|^2 = 2 per unit density), over 2 rho, minus
        // |u|^2 / 2
        T th = T(0);
        if constexpr (SS::TH) th = T(0.5) * ((ep - T(2) * rp) * inv - (ux * ux + uy * uy));
        // collision frequency p / mu: at a fixed viscosity it follows the
        // pressure p = rho T
        const T om = A.ph.tau_mode == TAU_RHO ? om_rho * rho * (T(1) + th) : om0;
        const T omr = om * rho, Gx = dtT * rho * gxT, Gy = dtT * rho * gyT;
        T px[EQ + 1], py[EQ + 1];
        hcoef<SS::TH>(ux, th, px);
        hcoef<SS::TH>(uy, th, py);
        // C_km: relaxation + force coefficient of He_k(x) He_m(y) / (k! m!):
        // the equilibrium's rho h_k(ux) h_m(uy) and the force's
        // k gx rho h_{k-1}(ux) h_m(uy) + m gy rho h_k(ux) h_{m-1}(uy)
        T C[EQ + 1][EQ + 1];
#pragma unroll
        for (int k = 0; k <= EQ; ++k)
#pragma unroll
            for (int m = 0; m + k <= EQ; ++m) {
                if (k == 0 && m == 0) {
                    C[0][0] = om * rp;
                } else {
                    T v = omr * px[k] * py[m];
                    if (k > 0) v += Gx * T(k) * px[k - 1] * py[m];
                    if (m > 0) v += Gy * T(m) * px[k] * py[m - 1];
                    C[k][m] = v;
                }
            }

#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const int q = q0 + qq;
            // B_k(q) = w_q sum_m C_km He_m(x_q)/m!
            T B[EQ + 1];
#pragma unroll
            for (int k = 0; k <= EQ; ++k) {
                T s = T(0);
#pragma unroll
                for (int m = 0; m + k <= EQ; ++m) s += C[k][m] * T(TB::rule.w[q] * TB::hk.v[m][q]);
                B[k] = s;
            }
            const double xq = TB::rule.x[q];
            T nq = T(0);
            T accq[N];   // this y-abscissa's updated values of the row
#pragma unroll
            for (int p = 0; p < N; ++p) {
                const int k = p + N * qq;
                const int a = p + N * q;
                const double xp = TB::rule.x[p];
                // source: (dt/tau) f_eq + dt g (shifted), separable in p and q
                T Sa = T(0);
#pragma unroll
                for (int kx = 0; kx <= EQ; ++kx) Sa += T(TB::rule.w[p] * TB::hk.v[kx][p]) * B[kx];
                const T f = c[k];
                // f - om f keeps the relaxation rate exact to FP32 rounding of om
                // ((1 - om) f would move it by eps/om relative)
                T acc = f - om * f + Sa;

                // x fluxes: neighbours from the adjacent lanes.  The limited
                // slope of column i, L_i = minmod(f_i - f_{i-1}, f_{i+1} - f_i),
                // is the one both faces need: the upwind face of column i
                // takes L_i and its neighbour's from the adjacent lane
                // (the same values as forming each face's slope in place)
                if (xp != 0.0) {
                    const T fm1 = xleft<WR>(f, col);
                    const T fp1 = xright<WR>(f, col);
                    const T dm = f - fm1, dp = fp1 - f;
                    const T L = minmod(dm, dp);
                    if (xp > 0.0) {
                        acc = acc - nu[p] * dm - kk[p] * (L - xleft<WR>(L, col));
                    } else {
                        acc = acc - nu[p] * dp - kk[p] * (xright<WR>(L, col) - L);
                    }
                }
                // y fluxes (register window)
                if (xq > 0.0) {
                    const T dp = nw[k] - f;
                    const T Lp = minmod(s1[k], dp);
                    acc = acc - nu[q] * s1[k] - kk[q] * (Lp - s2[k]);
                    c[k] = nw[k];
                    s1[k] = dp;
                    s2[k] = Lp;
                } else if (xq < 0.0) {
                    const T d = s1[k] - f, dn = nw[k] - s1[k];
                    const T Lp = minmod(dn, d);
                    acc = acc - nu[q] * d - kk[q] * (Lp - s2[k]);
                    c[k] = s1[k];
                    s1[k] = nw[k];
                    s2[k] = Lp;
                } else {
                    c[k] = nw[k];
                }
                // next row of this population (zero-cost past the strip end)
                nw[k] = LB_LD(a, LB_VO(vln, xq < 0.0 ? j + 3 : j + 2), LB_SO(a, xq < 0.0 ? j + 3 : j + 2));

                LB_ST(LB_VO(vs, j), LB_SO(a, j), acc)
                accq[p] = acc;
                // keep the scheduler from hoisting every population's
                // neighbour arithmetic to the top of the row (register blow-up)
                __builtin_amdgcn_sched_barrier(0);
            }
            // image columns and wall ghosts of this y-abscissa's populations:
            // one wave-uniform branch each per abscissa, not per population
            if (wave_img) {
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    const int a = p + N * q;
                    LB_ST(LB_VO(vimg_lo, j), LB_SO(a, j), accq[p])
                    LB_ST(LB_VO(vimg_hi, j), LB_SO(a, j), accq[p])
                }
            }
            if (wall) {
                // into the wall: bottom xi_y < 0, top xi_y > 0; those and
                // xi_y = 0 are final: copy them to the ghost rows
                const bool leaving = bottom ? (xq > 0.0) : (xq < 0.0);
                if (!leaving) {
#pragma unroll
                    for (int p = 0; p < N; ++p) {
                        const int a = p + N * q;
                        if (xq != 0.0) nq += T(lbt::cabs(xq)) * accq[p];
                        LB_ST(LB_VO(vw, gj1), LB_SO(a, gj1), accq[p])
                        LB_ST(LB_VO(vw, gj2), LB_SO(a, gj2), accq[p])
                    }
                }
            }
            if (wall) {
                if constexpr (SPLIT > 1) sn[bottom ? 0 : 1][q][lane] = nq;
                else nacc += nq;
            }
        }
        if (wall) {
            const int ws = bottom ? 0 : 1;
            if constexpr (SPLIT > 1) {
                __syncthreads();
#pragma unroll
                for (int q = 0; q < N; ++q) nacc += sn[ws][q][lane];
            }
            T Kw, Dw;
            if constexpr (sizeof(T) == 8) {
                Kw = A.ks.wK[ws];
                Dw = A.ks.wD[ws];
            } else {
                Kw = A.ks.wKf[ws];
                Dw = A.ks.wDf[ws];
            }
            const T d = (nacc - rho_shift * Dw) / (Kw + Dw);
#pragma unroll
            for (int k = 0; k < QW; ++k) {
                const int a = LB_POP(k);
                const double xq = TB::rule.x[q0 + k / N];
                if (xq == 0.0) continue;
                if (bottom != (xq > 0.0)) continue;   // leaving the wall only
                T sp;
                if constexpr (sizeof(T) == 8) sp = A.ks.sp[ws][a];
                else sp = A.ks.spf[ws][a];
                const T fl = d * T(TB::rule.w[a % N] * TB::rule.w[a / N]) + (d + rho_shift) * sp;
                const unsigned vil = NW ? (wall_l ? vimg_lo : OOB) : vimg_lo;
                const unsigned vih = NW ? (wall_l ? vimg_hi : OOB) : vimg_hi;
                LB_ST(LB_VO(vw, j), LB_SO(a, j), fl)
                LB_ST(LB_VO(vw, gj1), LB_SO(a, gj1), fl)
                LB_ST(LB_VO(vw, gj2), LB_SO(a, gj2), fl)
                if (wave_img) {
                    LB_ST(LB_VO(vil, j), LB_SO(a, j), fl)
                    LB_ST(LB_VO(vih, j), LB_SO(a, j), fl)
                }
            }
        }
    }
#undef LB_SOFF
#undef LB_VO
#undef LB_SO
#undef LB_POP
#undef LB_LD
}
#undef LB_ST

// order of the six components a tensor-product D2Q9 lacks at total order 3-4
__device__ __forceinline__ int missing_index(int k, int m) {
    if (k == 3 && m == 0) return 0;
    if (k == 0 && m == 3) return 1;
    if (k == 3 && m == 1) return 2;
    if (k == 1 && m == 3) return 3;
    if (k == 4 && m == 0) return 4;
    if (k == 0 && m == 4) return 5;
    return -1;
}


// Hermite-moment projection of one source node (set SS, absolute values
// fs) onto set DD (Sec. 2.2 in moment form), for the ND populations
// t = tp + ND tq of one target column tq; also returns rho, u of the node.
// The node's coefficients are formed once per column.
template <class SS, class DD>
__device__ void project_col(const double *fs, int tq, double *out, double &rho, double &ux, double &uy, double &th,
                            const float *cl6 = nullptr) {
    using TS = typename SS::T;
    using TD = typename DD::T;
    constexpr int NS = SS::N, ND = DD::N;
    constexpr int NM = NS < ND ? NS : ND;
    double tt[NS][NM];
#pragma unroll
    for (int p = 0; p < NS; ++p)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NS; ++q) s += fs[p + NS * q] * TS::he.v[m][q];
            tt[p][m] = s;
        }
    double a[NM][NM];
#pragma unroll
    for (int k = 0; k < NM; ++k)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            double s = 0.0;
#pragma unroll
            for (int p = 0; p < NS; ++p) s += TS::he.v[k][p] * tt[p][m];
            a[k][m] = s;
        }
    rho = a[0][0];
    ux = a[1][0] / rho;
    uy = a[0][1] / rho;
    th = SS::TH ? 0.5 * ((a[2][0] + a[0][2]) / rho - (ux * ux + uy * uy)) : 0.0;
    if constexpr (SS::N == DD::N && SS::EQ == DD::EQ) {
#pragma unroll
        for (int tp = 0; tp < ND; ++tp) out[tp] = fs[tp + ND * tq];
    } else {
        double px[ND + 1], py[ND + 1];
        hcoef<SS::TH>(ux, th, px);
        hcoef<SS::TH>(uy, th, py);
        double b[ND];
#pragma unroll
        for (int k = 0; k < ND; ++k) {
            double bk = 0.0;
#pragma unroll
            for (int m = 0; m < ND; ++m) {
                double eqd = (k + m <= DD::EQ) ? rho * px[k] * py[m] : 0.0;
                double neq = 0.0;
                if (k < NM && m < NM) {
                    neq = a[k][m] - ((k + m <= SS::EQ) ? rho * px[k] * py[m] : 0.0);
                } else if (cl6) {
                    const int mi = missing_index(k, m);
                    if (mi >= 0) neq = double(cl6[mi]);
                }
                bk += (eqd + neq) * TD::hk.v[m][tq];
            }
            b[k] = bk;
        }
#pragma unroll
        for (int tp = 0; tp < ND; ++tp) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) s += TD::hk.v[k][tp] * b[k];
            out[tp] = TD::rule.w[tp] * TD::rule.w[tq] * s;
        }
    }
}

// one population of the order-EQ equilibrium (absolute), temperature 1 + th
template <class SS>
__device__ double feq_one(double rho, double ux, double uy, double th, int t) {
    using TB = typename SS::T;
    const int tp = t % SS::N, tq = t / SS::N;
    double px[SS::EQ + 1], py[SS::EQ + 1];
    hcoef<SS::TH>(ux, th, px);
    hcoef<SS::TH>(uy, th, py);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k <= SS::EQ; ++k) {
        double b = 0.0;
#pragma unroll
        for (int m = 0; m + k <= SS::EQ; ++m) b += py[m] * TB::hk.v[m][tq];
        s += px[k] * TB::hk.v[k][tp] * b;
    }
    return TB::rule.w[tp] * TB::rule.w[tq] * rho * s;
}

// store one population t of set SS at node (i, j) and at every ghost entry
// standing for it (the per-population form of emit_node)
template <class ST, class SS>
__device__ void emit_pop(const Buf &b, int copy, int i, int j, const Shift &sh, int t, double v, double rho,
                         double ux, double uy, double th, const Geo &g, const Phys &ph) {
    typename ST::S *p0 = plane0<ST, SS>(b, copy) + (int64_t)t * b.plane;
    // absolute value x to entry (ii, jj), shifted by the reference of column ii
    auto put = [&](int ii, int jj, double x) {
        ST::std_(p0 + (int64_t)(jj + 2) * b.pitch + ii, x - w_of<SS>(t) * shift_at(sh, ii));
    };
    put(i, j, v);
    if (g.ybc == YBC_WALLS) {
        if (j == 0) { put(i, -1, v); put(i, -2, v); }
        if (j == g.ny) { put(i, g.ny + 1, v); put(i, g.ny + 2, v); }
    } else if (g.ybc == YBC_SHEAR) {
        if (j == 0) { put(i, -1, v); put(i, -2, v); }
        if (j == g.ny) {
            const double neq = v - feq_one<SS>(rho, ux, uy, th, t);
            put(i, g.ny + 1, feq_one<SS>(rho, ux + ph.shear, uy, th, t) + neq);
            put(i, g.ny + 2, feq_one<SS>(rho, ux + 2.0 * ph.shear, uy, th, t) + neq);
        }
    } else {
        if (j < 2) put(i, j + g.nrow, v);
        if (j >= g.nrow - 2) put(i, j - g.nrow, v);
    }
    if (g.xbc == XBC_PERIODIC) {
        if (i < 2) put(i + g.nx, j, v);
        if (i >= g.nx - 2) put(i - g.nx, j, v);
    } else if (i == 0 || i == g.nx - 1) {
        const double gv =
            feq_one<SS>(i == 0 ? ph.rho_in : ph.rho_out, ux, uy, th, t) + (v - feq_one<SS>(rho, ux, uy, th, t));
        if (i == 0) { put(-1, j, gv); put(-2, j, gv); }
        else { put(g.nx, j, gv); put(g.nx + 1, j, gv); }
    }
}

// Row images (periodic y) and pressure columns of the nodes listed in
// A.items (i, j, set, 0): node-local, from the freshly written copy, one
// thread per (node, population).
template <class ST, class LS, class HS>
__device__ __forceinline__ void finish_pop(const StepArgs &A, const int cur, const int i, const int j, const int set,
                                           const int t) {
    const int copy = cur ^ 1;
    double rho, ux, uy, th;
    if (set == 0) {
        if (t >= LS::Q) return;
        double f[LS::Q];
        load_node_d<ST, LS>(A.self, copy, i, j, sh_of(A), f);
        moments_td<LS>(f, rho, ux, uy, th);
        emit_pop<ST, LS>(A.self, copy, i, j, sh_of(A), t, f[t], rho, ux, uy, th, A.g, A.ph);
    } else {
        if (t >= HS::Q) return;
        double f[HS::Q];
        load_node_d<ST, HS>(A.other, copy, i, j, sh_of(A), f);
        moments_td<HS>(f, rho, ux, uy, th);
        emit_pop<ST, HS>(A.other, copy, i, j, sh_of(A), t, f[t], rho, ux, uy, th, A.g, A.ph);
    }
}

template <class LS, class HS>
constexpr int finish_qmax() { return LS::Q > HS::Q ? LS::Q : HS::Q; }

template <class ST, class LS, class HS>
__global__ __launch_bounds__(128) void k_finish(const StepArgs A) {
    constexpr int QM = finish_qmax<LS, HS>();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = k / QM;
    if (e >= A.nitems) return;
    finish_pop<ST, LS, HS>(A, A.cur, A.items[4 * e], A.items[4 * e + 1], A.items[4 * e + 2], k % QM);
}

// batch form: items (i, j, set, l)
template <class ST, class LS, class HS>
__global__ __launch_bounds__(128) void k_finish_batch(const BatchArgs B) {
    constexpr int QM = finish_qmax<LS, HS>();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int e = k / QM;
    if (e >= B.nitems) return;
    finish_pop<ST, LS, HS>(B.desc[B.items[4 * e + 3]], B.cur, B.items[4 * e], B.items[4 * e + 1], B.items[4 * e + 2],
                           k % QM);
}

// Hermite-moment projection of the halo-source nodes into the partner set,
// one thread per (node, target population).  A.items lists (i, j) pairs:
// the first A.nitems nodes of the low set project into the high set, the
// next A.chunk nodes of the high set into the low set.
// target column tq of the projection of node (i, j): up = low set into
// the high set (with the learned closure cl6 if given), else high into low
template <class ST, class LS, class HS>
__device__ __forceinline__ void project_entry(const StepArgs &A, const int cur, const bool up, const int i,
                                              const int j, const int tq, const float *cl6) {
    const int copy = cur ^ 1;
    double rho, ux, uy, th;
    if (up) {
        double fs[LS::Q], out[HS::N];
        load_node_d<ST, LS>(A.self, copy, i, j, sh_of(A), fs);
        project_col<LS, HS>(fs, tq, out, rho, ux, uy, th, cl6);
#pragma unroll
        for (int tp = 0; tp < HS::N; ++tp)
            emit_pop<ST, HS>(A.other, copy, i, j, sh_of(A), tp + HS::N * tq, out[tp], rho, ux, uy, th, A.g, A.ph);
    } else {
        double fs[HS::Q], out[LS::N];
        load_node_d<ST, HS>(A.other, copy, i, j, sh_of(A), fs);
        project_col<HS, LS>(fs, tq, out, rho, ux, uy, th);
#pragma unroll
        for (int tp = 0; tp < LS::N; ++tp)
            emit_pop<ST, LS>(A.self, copy, i, j, sh_of(A), tp + LS::N * tq, out[tp], rho, ux, uy, th, A.g, A.ph);
    }
}

// thread k of the projection pass: one per (node, target column)
template <class ST, class LS, class HS>
__device__ __forceinline__ void project_halo_thread(const StepArgs &A, const int64_t k) {
    const int64_t n0 = (int64_t)A.nitems * HS::N, n1 = (int64_t)A.chunk * LS::N;
    if (k < n0) {
        const int e = int(k / HS::N), tq = int(k % HS::N);
        project_entry<ST, LS, HS>(A, A.cur, true, A.items[2 * e], A.items[2 * e + 1], tq,
                                  A.clo ? A.clo + 6 * e : nullptr);
    } else if (k < n0 + n1) {
        const int e = int((k - n0) / LS::N) + A.nitems, tq = int((k - n0) % LS::N);
        project_entry<ST, LS, HS>(A, A.cur, false, A.items[2 * e], A.items[2 * e + 1], tq, nullptr);
    }
}

template <class ST, class LS, class HS>
__global__ __launch_bounds__(128) void k_project_halo(const StepArgs A) {
    project_halo_thread<ST, LS, HS>(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The projection and finish passes of one step in one launch: blocks below
// nbp project (as k_project_halo), the rest finish the nodes of `fin` (as
// k_finish).  Both read only the updated copy, and their writes are
// disjoint: a projection writes the partner set's entries of a node and
// their ghosts/images, the finish pass a node's own set's ghosts, images and
// pressure columns, and no node belongs to both sets.
template <class ST, class LS, class HS>
__global__ __launch_bounds__(128) void k_project_finish(const StepArgs A, const int32_t *fin, const int nfin,
                                                        const int nbp) {
    if ((int)blockIdx.x < nbp) {
        project_halo_thread<ST, LS, HS>(A, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
        return;
    }
    constexpr int QM = finish_qmax<LS, HS>();
    const int k = ((int)blockIdx.x - nbp) * blockDim.x + threadIdx.x;
    const int e = k / QM;
    if (e >= nfin) return;
    finish_pop<ST, LS, HS>(A, A.cur, fin[4 * e], fin[4 * e + 1], fin[4 * e + 2], k % QM);
}

// batch form: items (i, j, l, 0) of lattice l, whose arguments (self = low
// set) are desc[l]; the first nup entries project up, the next ndown down;
// one thread per (node, target column), k counted from the slot's first
// block
template <class ST, class LS, class HS>
__device__ __forceinline__ void project_batch_entry(const StepArgs *desc, const int32_t *items, const int nup,
                                                    const int ndown, const int cur, const int64_t k) {
    const int64_t n0 = (int64_t)nup * HS::N, n1 = (int64_t)ndown * LS::N;
    int e, tq;
    bool up;
    if (k < n0) {
        e = int(k / HS::N);
        tq = int(k % HS::N);
        up = true;
    } else if (k < n0 + n1) {
        e = int((k - n0) / LS::N) + nup;
        tq = int((k - n0) % LS::N);
        up = false;
    } else {
        return;
    }
    project_entry<ST, LS, HS>(desc[items[4 * e + 2]], cur, up, items[4 * e], items[4 * e + 1], tq, nullptr);
}

// one set pair per launch (pairs outside the three slots of k_project_multi)
template <class ST, class LS, class HS>
__global__ __launch_bounds__(128) void k_project_halo_batch(const BatchArgs B) {
    project_batch_entry<ST, LS, HS>(B.desc, B.items, B.nitems, B.nsplit, B.cur,
                                    (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// the pairs D2Q9/D2Q36, D2Q16/D2Q36 and D2Q9/D2Q16 in one launch
template <class ST, class S36, class S16>
__global__ __launch_bounds__(128) void k_project_multi(const BatchMulti M) {
    using S9 = lbt::VSet<3, 2>;
    const int b = blockIdx.x;
    const int t = threadIdx.x;
    if (b < M.start[1])
        project_batch_entry<ST, S9, S36>(M.desc, M.items[0], M.nitems[0], M.nsplit[0], M.cur, (int64_t)b * 128 + t);
    else if (b < M.start[2])
        project_batch_entry<ST, S16, S36>(M.desc, M.items[1], M.nitems[1], M.nsplit[1], M.cur,
                                          (int64_t)(b - M.start[1]) * 128 + t);
    else
        project_batch_entry<ST, S9, S16>(M.desc, M.items[2], M.nitems[2], M.nsplit[2], M.cur,
                                         (int64_t)(b - M.start[2]) * 128 + t);
}

// ---------------------------------------------------- persistent batch
// One launch advances every lattice of a batch by P.nsteps steps.  Work-
// group b owns the lattices P.wl[P.wl_off[b] .. P.wl_off[b + 1]) -- whole
// lattices, assigned by the host largest-first by populations x nodes --
// and loops over the steps with workgroup barriers only; no workgroup waits
// on another.  Each update item runs on one wave holding all of its
// populations (split over waves, an item would carry a barrier per row, and
// waves could not take different items); the PERSIST_WAVES waves take a
// lattice's items in turn, then, after a barrier, every thread takes the
// lattice's projection entries in turn, and a barrier closes the step.  A
// node's update and projection are the same arithmetic as in the other
// launches, so the results are bit-identical to lb_step.
constexpr int PERSIST_WAVES = 8;

__device__ __forceinline__ uint32_t step_seed_dev(int64_t n) {
    return uint32_t(uint64_t(n) * 0x9e3779b97f4a7c15ull >> 32);
}

// one update item of set SS on a single wave (i0 encodes the item shape as
// for the batch update: wide, narrow lane groups, or wrapped 8-column groups)
template <class ST, class SS>
__device__ __forceinline__ void persist_item(const StepArgs &A, const int cur, const uint32_t seed, const int i0,
                                             const int j0, const int j1) {
    if (i0 <= -NW_WRAP) update_item<ST, SS, SS, true, 1, true>(A, cur, seed, 0, j0, j1, -i0 - NW_WRAP);
    else if (i0 < 0) update_item<ST, SS, SS, true, 1>(A, cur, seed, 0, j0, j1, -i0);
    else update_item<ST, SS, SS, false, 1>(A, cur, seed, i0, j0, j1);
}

template <class ST, class S36, class S16>
__global__ __launch_bounds__(64 * PERSIST_WAVES) __attribute__((amdgpu_waves_per_eu(2)))
void k_batch_persistent(const PersistArgs P) {
    using S9 = lbt::VSet<3, 2>;
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const int b = blockIdx.x;
    const int l0 = P.wl_off[b], l1 = P.wl_off[b + 1];
    for (int s = 0; s < P.nsteps; ++s) {
        const int cur = P.cur ^ (s & 1);
        const uint32_t seed = step_seed_dev(P.step0 + s);
        for (int li = l0; li < l1; ++li) {
            const int32_t *m = P.lat + 8 * P.wl[li];
            const int ioff = __builtin_amdgcn_readfirstlane(m[0]), nit = __builtin_amdgcn_readfirstlane(m[1]);
            for (int it = w; it < nit; it += PERSIST_WAVES) {
                const int32_t *e = P.items + 4 * (ioff + it);
                const int i0 = __builtin_amdgcn_readfirstlane(e[0]);
                const int j0 = __builtin_amdgcn_readfirstlane(e[1]);
                const int j1 = __builtin_amdgcn_readfirstlane(e[2]);
                const int code = __builtin_amdgcn_readfirstlane(e[3]);
                if (j0 >= j1) continue;
                const StepArgs &A =
                    *(const StepArgs *)((const __attribute__((address_space(4))) StepArgs *)P.desc + (code & 0x0fffffff));
                const int kind = code >> 28;
                if (kind == 0) persist_item<ST, S36>(A, cur, seed, i0, j0, j1);
                else if (kind == 1) persist_item<ST, S16>(A, cur, seed, i0, j0, j1);
                else persist_item<ST, S9>(A, cur, seed, i0, j0, j1);
            }
        }
        __syncthreads();   // every update of this workgroup's lattices is written
        for (int li = l0; li < l1; ++li) {
            const int32_t *m = P.lat + 8 * P.wl[li];
            const int32_t *pe = P.proj + 4 * m[2];
            const int nup = m[3], ndown = m[4], pair = m[5];
            if (pair == 0) {
                const int64_t n = int64_t(nup) * S36::N + int64_t(ndown) * S9::N;
                for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
                    project_batch_entry<ST, S9, S36>(P.desc, pe, nup, ndown, cur, k);
            } else if (pair == 1) {
                const int64_t n = int64_t(nup) * S36::N + int64_t(ndown) * S16::N;
                for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
                    project_batch_entry<ST, S16, S36>(P.desc, pe, nup, ndown, cur, k);
            } else if (pair == 2) {
                const int64_t n = int64_t(nup) * S16::N + int64_t(ndown) * S9::N;
                for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
                    project_batch_entry<ST, S9, S16>(P.desc, pe, nup, ndown, cur, k);
            }
        }
        __syncthreads();   // the halos are written before the next step reads them
    }
}

// ------------------------------------------------------- learned closure
// (the kernel that runs the closure inside the projection launch,
// k_project_closure, follows the inference kernel below)
// Network 10 -> 64 -> 64 -> 8 (tanh, tanh, linear); parameter layout
// W1[64][10], b1[64], W2[64][64], b2[64], W3[8][64], b3[8].
constexpr int MLP_NIN = 10, MLP_NH = 64, MLP_NOUT = 8;
constexpr int MLP_OFF_B1 = MLP_NH * MLP_NIN, MLP_OFF_W2 = MLP_OFF_B1 + MLP_NH;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_NH * MLP_NH, MLP_OFF_W3 = MLP_OFF_B2 + MLP_NH;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_NOUT * MLP_NH, MLP_NPARAM = MLP_OFF_B3 + MLP_NOUT;

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ uint16_t f_to_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// Raw inputs of a D2Q9 node (absolute populations): rho - 1, ux, uy,
// log Kn_loc, then (a_km - a_eq,km)/rho for (2,0),(1,1),(0,2),(2,1),(1,2),(2,2)
// with the 2nd-order equilibrium (no components above order 2).
template <class LS>
__device__ void closure_features(const double *f9, double kn_loc, double &rho, float *x) {
    using TL = typename LS::T;
    double a[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double s = 0.0;
#pragma unroll
            for (int al = 0; al < 9; ++al) s += f9[al] * TL::he.v[k][al % 3] * TL::he.v[m][al / 3];
            a[k][m] = s;
        }
    rho = a[0][0];
    const double ux = a[1][0] / rho, uy = a[0][1] / rho;
    x[0] = float(rho - 1.0);
    x[1] = float(ux);
    x[2] = float(uy);
    x[3] = float(log(kn_loc));
    x[4] = float((a[2][0] - rho * ux * ux) / rho);
    x[5] = float((a[1][1] - rho * ux * uy) / rho);
    x[6] = float((a[0][2] - rho * uy * uy) / rho);
    x[7] = float(a[2][1] / rho);
    x[8] = float(a[1][2] / rho);
    x[9] = float(a[2][2] / rho);
}

// FP32 forward pass with bf16 weights (bits in w); x standardised in place
template <class W>
__device__ void mlp_forward_one(const W &w, const float *x, float *y) {
    float h1[MLP_NH];
#pragma unroll 4
    for (int o = 0; o < MLP_NH; ++o) {
        float s = w(MLP_OFF_B1 + o);
#pragma unroll
        for (int k = 0; k < MLP_NIN; ++k) s += w(o * MLP_NIN + k) * x[k];
        h1[o] = tanhf(s);
    }
    float h2[MLP_NH];
    for (int o = 0; o < MLP_NH; ++o) {
        float s = w(MLP_OFF_B2 + o);
#pragma unroll 8
        for (int k = 0; k < MLP_NH; ++k) s += w(MLP_OFF_W2 + o * MLP_NH + k) * h1[k];
        h2[o] = tanhf(s);
    }
#pragma unroll
    for (int o = 0; o < MLP_NOUT; ++o) {
        float s = w(MLP_OFF_B3 + o);
#pragma unroll 8
        for (int k = 0; k < MLP_NH; ++k) s += w(MLP_OFF_W3 + o * MLP_NH + k) * h2[k];
        y[o] = s;
    }
}

struct WBf16 {
    const uint16_t *p;
    __device__ float operator()(int i) const { return bf16_to_f(p[i]); }
};

// closure coefficients C_km of the six missing components for one D2Q9 node
template <class LS, class W>
__device__ void closure_coeffs(const W &w, const ClosureNorm &cn, const double *f9, double rho_ref, float *c6) {
    float x[MLP_NIN], y[MLP_NOUT];
    double rho;
    // local Kn: Kn at rho_ref, scaled as 1/rho when the relaxation time is
    double a00 = 0.0;
#pragma unroll
    for (int al = 0; al < 9; ++al) a00 += f9[al];
    const double kn_loc = cn.tau_rho ? cn.kn_ref * rho_ref / a00 : cn.kn_ref;
    closure_features<LS>(f9, kn_loc, rho, x);
#pragma unroll
    for (int k = 0; k < MLP_NIN; ++k) x[k] = (x[k] - cn.xmean[k]) / cn.xstd[k];
    mlp_forward_one(w, x, y);
#pragma unroll
    for (int k = 0; k < 6; ++k) c6[k] = float(rho) * (cn.tmean[k] + cn.tstd[k] * y[k]);
}

// The network on the matrix cores: one wave evaluates 16 nodes with
// v_mfma_f32_16x16x16_bf16 tiles (nodes x hidden units), weights as their
// bf16 bits, FP32 accumulation.  Inputs and activations enter as two bf16
// terms (hi + lo, 16 significant bits together), so the result carries the
// FP32 network's accuracy rather than bf16 activations'.  Operand layouts
// (16 x 16 x 16): A[i][k] in lane i + 16 (k / 4), element k % 4; B[k][j] in
// lane j + 16 (k / 4), element k % 4; D[i][j] in lane j + 16 (i / 4),
// register i % 4.
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// tanh of the inference layers: 1 - 2 / (exp(2|x|) + 1) with the
// hardware exponential and reciprocal, sign restored (absolute error about
// 1e-7, inside the 16 significant bits the next layer takes; for large |x|
// the exponential overflows to infinity and the result is exactly 1)
__device__ __forceinline__ float tanh_fast(float x) {
    const float e = __expf(2.0f * fabsf(x));
    return copysignf(1.0f - __fdividef(2.0f, e + 1.0f), x);
}

__device__ __forceinline__ void bf16_split(float v, short &hi, short &lo) {
    const uint16_t h = f_to_bf16(v);
    hi = short(h);
    lo = short(f_to_bf16(v - bf16_to_f(h)));
}

// xs: standardised inputs of the 16 nodes (K padded to 16 with zeros);
// hs: LDS scratch [16][64 + 4]; out: c6 of the 16 nodes (rho * (mean + std y))
// and, when zf is given, the two region-flag logits of each node
__device__ __forceinline__ void closure_mfma16(const uint16_t *w, const ClosureNorm &cn, const float (*xs)[16],
                                               float (*hs)[MLP_NH + 4], const float *rs, float (*c6)[6],
                                               float (*zf)[2] = nullptr) {
    const int l = threadIdx.x & 63;
    const int r = l & 15, kq = l >> 4;
    const f32x4_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4_t acc[4];
    // layer 1: [16 nodes x 16 inputs] x [16 x 64]
    bf16x4_t ah, al;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        short h, lo;
        bf16_split(xs[r][4 * kq + e], h, lo);
        ah[e] = h;
        al[e] = lo;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x4_t b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = 4 * kq + e;
            b[e] = k < MLP_NIN ? short(w[(16 * t + r) * MLP_NIN + k]) : short(0);
        }
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, b, zero, 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, b, acc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float b1 = bf16_to_f(w[MLP_OFF_B1 + 16 * t + r]);
#pragma unroll
        for (int v = 0; v < 4; ++v) hs[4 * kq + v][16 * t + r] = tanh_fast(acc[t][v] + b1);
    }
    __syncthreads();
    // layers 2 and 3: [16 x 64] x [64 x 64], then [16 x 64] x [64 x 16 (8 used)]
#pragma unroll
    for (int layer = 2; layer <= 3; ++layer) {
        const int nt = layer == 2 ? 4 : 1;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = zero;
#pragma unroll
        for (int sk = 0; sk < 4; ++sk) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                short h, lo;
                bf16_split(hs[r][16 * sk + 4 * kq + e], h, lo);
                ah[e] = h;
                al[e] = lo;
            }
#pragma unroll
            for (int t = 0; t < nt; ++t) {
                bf16x4_t b;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 16 * sk + 4 * kq + e;
                    if (layer == 2) b[e] = short(w[MLP_OFF_W2 + (16 * t + r) * MLP_NH + k]);
                    else b[e] = r < MLP_NOUT ? short(w[MLP_OFF_W3 + r * MLP_NH + k]) : short(0);
                }
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, b, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, b, acc[t], 0, 0, 0);
            }
        }
        __syncthreads();   // every lane has read the previous activations
        if (layer == 2) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float b2 = bf16_to_f(w[MLP_OFF_B2 + 16 * t + r]);
#pragma unroll
                for (int v = 0; v < 4; ++v) hs[4 * kq + v][16 * t + r] = tanh_fast(acc[t][v] + b2);
            }
            __syncthreads();
        } else if (r < 6) {
            const float b3 = bf16_to_f(w[MLP_OFF_B3 + r]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int n = 4 * kq + v;
                c6[n][r] = rs[n] * (cn.tmean[r] + cn.tstd[r] * (acc[0][v] + b3));
            }
        } else if (r < MLP_NOUT && zf) {
            const float b3 = bf16_to_f(w[MLP_OFF_B3 + r]);
#pragma unroll
            for (int v = 0; v < 4; ++v) zf[4 * kq + v][r - 6] = acc[0][v] + b3;
        }
    }
    __syncthreads();
}

// the network's bf16 weights copied to LDS by the block's threads in
// 16-byte pieces (the layers then read their operands from LDS instead of
// issuing two-byte global loads on the critical path); the caller's next
// barrier publishes them
static_assert(MLP_NPARAM * 2 % 16 == 0, "weights copy in 16-byte pieces");
__device__ __forceinline__ void stage_closure_weights(const uint16_t *w, uint16_t *wl) {
    const uint4 *src = reinterpret_cast<const uint4 *>(w);
    uint4 *dst = reinterpret_cast<uint4 *>(wl);
    for (int k = threadIdx.x; k < MLP_NPARAM * 2 / 16; k += blockDim.x) dst[k] = src[k];
}

// standardised inputs and density of one D2Q9 node (absolute populations)
template <class LS>
__device__ __forceinline__ void closure_inputs(const ClosureNorm &cn, const double *f9, double rho_ref, float *xs16,
                                               float &rho_out) {
    double a00 = 0.0;
#pragma unroll
    for (int al = 0; al < 9; ++al) a00 += f9[al];
    // local Kn: Kn at rho_ref, scaled as 1/rho when the relaxation time is
    const double kn_loc = cn.tau_rho ? cn.kn_ref * rho_ref / a00 : cn.kn_ref;
    double rho;
    float x[MLP_NIN];
    closure_features<LS>(f9, kn_loc, rho, x);
#pragma unroll
    for (int k = 0; k < 16; ++k) xs16[k] = k < MLP_NIN ? (x[k] - cn.xmean[k]) / cn.xstd[k] : 0.0f;
    rho_out = float(rho);
}

// Per step, before the projection pass: closure coefficients of the lifted
// nodes (the first A.nitems entries of the projection list, low set), one
// wave per CLOSURE_NB = 16 nodes.
template <class ST, class LS, class HS>
__global__ __launch_bounds__(64) void k_closure_infer(const StepArgs A) {
    if constexpr (LS::N == 3 && HS::N == 6 && !LS::TH) {
        __shared__ float xs[16][16];
        __shared__ float hs[16][MLP_NH + 4];
        __shared__ float rs[16];
        __shared__ float c6[16][6];
        __shared__ __attribute__((aligned(16))) uint16_t wl[MLP_NPARAM];
        const int lane = threadIdx.x;
        const int e0 = blockIdx.x * CLOSURE_NB;
        const int nn = min(CLOSURE_NB, A.nitems - e0);
        stage_closure_weights(A.clw, wl);
        if (lane < 16) {
            if (lane < nn) {
                const int e = e0 + lane;
                const int i = A.items[2 * e], j = A.items[2 * e + 1];
                double f9[9];
                load_node_d<ST, LS>(A.self, A.cur ^ 1, i, j, sh_of(A), f9);
                closure_inputs<LS>(A.cn, f9, A.ph.rho_ref, xs[lane], rs[lane]);
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k) xs[lane][k] = 0.0f;
                rs[lane] = 0.0f;
            }
        }
        __syncthreads();
        closure_mfma16(wl, A.cn, xs, hs, rs, c6);
        for (int q = lane; q < 6 * nn; q += 64) A.clo[6 * e0 + q] = c6[q / 6][q % 6];
    }
}

// The network's region flag of every node, beside the indicator: a node
// whose flag logits favour the high-order set (z1 > z0) gets an indicator of
// +infinity in B, so the band rule keeps it in the high set whatever the
// threshold.  Inputs come from the node's D2Q9 populations, or from its
// D2Q36 populations restricted to D2Q9 (Hermite projection) in the high
// bands; one wave per 16 nodes, row-major.  self = low set, other = high.
// A learned-closure step's inference, projection and finish pass in one
// launch (one wave per block), instead of the inference launch before the
// projection launch.  Blocks below nbl take 16 lifted nodes each: the
// network's outputs stay in LDS and the same wave then projects those
// nodes into the high set (6 target columns each), as k_project_halo does
// with the outputs k_closure_infer stores; the next nbd blocks project the
// high set's halo sources down (64 entries each), the remaining blocks
// finish the nodes of `fin` (one thread per node and population).  The
// three parts write disjoint entries and read only the updated copy.
template <class ST, class LS, class HS>
__global__ __launch_bounds__(64) void k_project_closure(const StepArgs A, const int32_t *fin, const int nfin,
                                                        const int nbl, const int nbd) {
    if constexpr (LS::N == 3 && HS::N == 6 && !LS::TH) {
        const int b = blockIdx.x, lane = threadIdx.x;
        if (b < nbl) {
            __shared__ float xs[16][16];
            __shared__ float hs[16][MLP_NH + 4];
            __shared__ float rs[16];
            __shared__ float c6[16][6];
            __shared__ __attribute__((aligned(16))) uint16_t wl[MLP_NPARAM];
            const int e0 = b * CLOSURE_NB;
            const int nn = min(CLOSURE_NB, A.nitems - e0);
            stage_closure_weights(A.clw, wl);
            if (lane < 16) {
                if (lane < nn) {
                    const int e = e0 + lane;
                    double f9[9];
                    load_node_d<ST, LS>(A.self, A.cur ^ 1, A.items[2 * e], A.items[2 * e + 1], sh_of(A), f9);
                    closure_inputs<LS>(A.cn, f9, A.ph.rho_ref, xs[lane], rs[lane]);
                } else {
#pragma unroll
                    for (int k = 0; k < 16; ++k) xs[lane][k] = 0.0f;
                    rs[lane] = 0.0f;
                }
            }
            __syncthreads();
            closure_mfma16(wl, A.cn, xs, hs, rs, c6);   // ends with a barrier: c6 is complete
            for (int k = lane; k < HS::N * nn; k += 64) {
                const int n = k / HS::N, e = e0 + n;
                project_entry<ST, LS, HS>(A, A.cur, true, A.items[2 * e], A.items[2 * e + 1], k % HS::N, c6[n]);
            }
            return;
        }
        if (b < nbl + nbd) {
            const int64_t k = int64_t(b - nbl) * 64 + lane;
            if (k >= int64_t(A.chunk) * LS::N) return;
            const int e = int(k / LS::N) + A.nitems;
            project_entry<ST, LS, HS>(A, A.cur, false, A.items[2 * e], A.items[2 * e + 1], int(k % LS::N), nullptr);
            return;
        }
        constexpr int QM = finish_qmax<LS, HS>();
        const int k = (b - nbl - nbd) * 64 + lane;
        const int e = k / QM;
        if (e >= nfin) return;
        finish_pop<ST, LS, HS>(A, A.cur, fin[4 * e], fin[4 * e + 1], fin[4 * e + 2], k % QM);
    }
}

template <class ST, class LS, class HS>
__global__ __launch_bounds__(64) void k_closure_flags(const NodeArgs A) {
    if constexpr (LS::N == 3 && HS::N == 6 && !LS::TH) {
        __shared__ float xs[16][16];
        __shared__ float hs[16][MLP_NH + 4];
        __shared__ float rs[16];
        __shared__ float c6[16][6];
        __shared__ float zf[16][2];
        __shared__ __attribute__((aligned(16))) uint16_t wl[MLP_NPARAM];
        const int lane = threadIdx.x;
        const int64_t nodes = int64_t(A.g.nx) * A.g.nrow;
        const int64_t e0 = int64_t(blockIdx.x) * 16;
        const int nn = int(min(int64_t(16), nodes - e0));
        stage_closure_weights(A.clw, wl);
        if (lane < 16) {
            if (lane < nn) {
                const int64_t e = e0 + lane;
                const int j = int(e / A.g.nx), i = int(e - int64_t(j) * A.g.nx);
                double f9[9];
                if (region_at(i, j, A.g) == REG_HIGH) {
                    double f36[36];
                    load_node_d<ST, HS>(A.other, A.cur, i, j, sh_of(A), f36);
                    project_d<HS, LS>(f36, f9, nullptr);
                } else {
                    load_node_d<ST, LS>(A.self, A.cur, i, j, sh_of(A), f9);
                }
                closure_inputs<LS>(A.cn, f9, A.ph.rho_ref, xs[lane], rs[lane]);
            } else {
#pragma unroll
                for (int k = 0; k < 16; ++k) xs[lane][k] = 0.0f;
                rs[lane] = 0.0f;
            }
        }
        __syncthreads();
        closure_mfma16(wl, A.cn, xs, hs, rs, c6, zf);
        if (lane < nn && zf[lane][1] > zf[lane][0]) A.out0[e0 + lane] = __builtin_huge_val();
    }
}

// Training samples from the high set of an all-high run: for each listed
// node, raw features of its restriction to the low set, raw regression
// targets (missing non-equilibrium coefficients / rho) and the flag
// (indicator above theta).
template <class ST, class HS, class LS>
__global__ void k_closure_samples(const NodeArgs A) {
    if constexpr (LS::N == 3 && HS::N == 6 && !LS::TH) {
        const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (k >= A.nnodes) return;
        const int n = A.nodes[k];
        if (n < 0 || n >= A.g.nx * A.g.nrow) {   // not a node: marked, nothing read
            for (int q = 0; q < MLP_NIN; ++q) A.fx[MLP_NIN * k + q] = __builtin_nanf("");
            for (int q = 0; q < 6; ++q) A.ft[6 * k + q] = __builtin_nanf("");
            A.flag[k] = -1;
            return;
        }
        const int j = n / A.g.nx, i = n - j * A.g.nx;
        using TH = typename HS::T;
        double f36[36], f9[9];
        load_node_d<ST, HS>(A.self, A.cur, i, j, sh_of(A), f36);
        project_d<HS, LS>(f36, f9, nullptr);
        double a[6][6];
#pragma unroll
        for (int kk = 0; kk < 6; ++kk)
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                if (kk > 4 || m > 4) continue;
                double s = 0.0;
#pragma unroll
                for (int al = 0; al < 36; ++al) s += f36[al] * TH::he.v[kk][al % 6] * TH::he.v[m][al / 6];
                a[kk][m] = s;
            }
        const double rho = a[0][0], ux = a[1][0] / rho, uy = a[0][1] / rho;
        auto neq = [&](int kk, int m) {
            double eq = 1.0;
            for (int q = 0; q < kk; ++q) eq *= ux;
            for (int q = 0; q < m; ++q) eq *= uy;
            return (a[kk][m] - (kk + m <= HS::EQ ? rho * eq : 0.0)) / rho;
        };
        float *t = A.ft + 6 * k;
        t[0] = float(neq(3, 0));
        t[1] = float(neq(0, 3));
        t[2] = float(neq(3, 1));
        t[3] = float(neq(1, 3));
        t[4] = float(neq(4, 0));
        t[5] = float(neq(0, 4));
        const double b = fmax(fabs(neq(2, 0)), fmax(fabs(neq(1, 1)), fabs(neq(0, 2))));
        A.flag[k] = b > A.theta ? 1 : 0;
        // local Kn: Kn at rho_ref, scaled as 1/rho when the relaxation time is
        const double kn_loc = A.ph.tau_mode == TAU_RHO ? A.ph.kn * A.ph.rho_ref / rho : A.ph.kn;
        double r9;
        float x[MLP_NIN];
        closure_features<LS>(f9, kn_loc, r9, x);
#pragma unroll
        for (int q = 0; q < MLP_NIN; ++q) A.fx[MLP_NIN * k + q] = x[q];
    }
}

// ------------------------------------------------------ per-node kernels
__device__ __forceinline__ bool node_index(const Geo &g, int &i, int &j) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.nrow * g.nx) return false;
    j = n / g.nx;
    i = n - j * g.nx;
    return true;
}

__device__ __forceinline__ bool owns(int r, bool self_high) {
    return self_high ? r == REG_HIGH : r == REG_LOW;
}

// Rebuild all ghost, image and projection entries of copy `cur` from the
// nodes' own entries (after initialisation, set_populations or a region
// change).
template <class ST, class SS, class OO>
__global__ void k_refresh(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!owns(r, A.self_high)) return;
    double f[SS::Q];
    load_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
    int t = tile_of(i, A.g);
    bool proj = (OO::Q > 0) && A.g.iface == IF_HERMITE &&
                neighbour_in(i, j, A.self_high ? REG_LOW : REG_HIGH, A.g.blo[t], A.g.bhi[t], A.g);
    finish_node<ST, SS, OO>(A.self, A.other, A.cur, i, j, sh_of(A), f, false, proj, A.g, A.ph);
}

// f = f_eq(rho, u, T) on the nodes of this set (in0..3 = rho, ux, uy, T
// fields; T only on thermal sets, NULL = 1)
template <class ST, class SS, class OO>
__global__ void k_init_eq(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!owns(r, A.self_high)) return;
    int n = j * A.g.nx + i;
    double f[SS::Q];
    const double th = (SS::TH && A.in3) ? A.in3[n] - 1.0 : 0.0;
    feq_d<SS>(A.in0[n], A.in1[n], A.in2[n], th, f);
    store_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
}

// populations from an FP64 [Q][nrow][nx] array (own nodes and, for the low
// set in the paper interface mode, the interface rows; the high set stores
// interface rows too)
template <class ST, class SS, class OO>
__global__ void k_set_pop(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!owns(r, A.self_high) && r != REG_IFACE) return;
    const int64_t NN = (int64_t)A.g.nrow * A.g.nx;
    double f[SS::Q];
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) f[a] = A.in0[a * NN + j * A.g.nx + i];
    store_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
}

template <class ST, class SS, class OO>
__global__ void k_get_pop(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    const int64_t NN = (int64_t)A.g.nrow * A.g.nx;
    double f[SS::Q];
    if (owns(r, A.self_high) || r == REG_IFACE) {
        load_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
    } else {
#pragma unroll
        for (int a = 0; a < SS::Q; ++a) f[a] = __builtin_nan("");
    }
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) A.out0[a * NN + j * A.g.nx + i] = f[a];
}

// rho, ux, uy of the nodes of this set (the low set also reports the
// interface rows, whose representations all carry rho_I, u_I)
template <class ST, class SS, class OO>
__global__ void k_moments(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!(owns(r, A.self_high) || (!A.self_high && r == REG_IFACE))) return;
    double f[SS::Q], rho, ux, uy;
    load_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
    moments_d<SS>(f, rho, ux, uy);
    int n = j * A.g.nx + i;
    A.out0[n] = rho;
    A.out1[n] = ux;
    A.out2[n] = uy;
}

// Thermal state of a node from its raw moments M1 = sum xi f,
// M2_ij = sum xi_i xi_j f, M3_i = sum xi_i |xi|^2 f: rho, u, T = tr P / (2 rho)
// with P_ij = M2_ij - rho u_i u_j, and the heat flux
// q_i = 1/2 sum c_i |c|^2 f = (M3_i - 2 u_j M2_ij - u_i tr M2 + 2 rho u_i |u|^2) / 2
// (c = xi - u expanded).
struct ThermalState {
    double rho, ux, uy, T, pxx, pxy, pyy, qx, qy;
};
template <class SS>
__device__ ThermalState thermal_state(const double *f) {
    using TB = typename SS::T;
    constexpr int N = SS::N;
    double m0 = 0, mx = 0, my = 0, mxx = 0, mxy = 0, myy = 0, m3x = 0, m3y = 0;
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) {
        const double x = TB::rule.x[a % N], y = TB::rule.x[a / N], x2 = x * x + y * y;
        m0 += f[a];
        mx += x * f[a];
        my += y * f[a];
        mxx += x * x * f[a];
        mxy += x * y * f[a];
        myy += y * y * f[a];
        m3x += x * x2 * f[a];
        m3y += y * x2 * f[a];
    }
    ThermalState t;
    t.rho = m0;
    t.ux = mx / m0;
    t.uy = my / m0;
    t.pxx = mxx - m0 * t.ux * t.ux;
    t.pxy = mxy - m0 * t.ux * t.uy;
    t.pyy = myy - m0 * t.uy * t.uy;
    t.T = 0.5 * (t.pxx + t.pyy) / m0;
    const double u2 = t.ux * t.ux + t.uy * t.uy, tr = mxx + myy;
    t.qx = 0.5 * (m3x - 2.0 * (t.ux * mxx + t.uy * mxy) - t.ux * tr + 2.0 * m0 * t.ux * u2);
    t.qy = 0.5 * (m3y - 2.0 * (t.ux * mxy + t.uy * myy) - t.uy * tr + 2.0 * m0 * t.uy * u2);
    return t;
}

// Temperature and heat flux (qx, qy) of the nodes of this set (out0..2);
// with A.mode = 1, the energy density 1/2 sum |xi|^2 f into out0 instead.
template <class ST, class SS, class OO>
__global__ void k_thermal(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!(owns(r, A.self_high) || (!A.self_high && r == REG_IFACE))) return;
    double f[SS::Q];
    load_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
    const ThermalState t = thermal_state<SS>(f);
    const int n = j * A.g.nx + i;
    if (A.mode == 1) {
        A.out0[n] = 0.5 * (t.pxx + t.pyy) + 0.5 * t.rho * (t.ux * t.ux + t.uy * t.uy);
        return;
    }
    A.out0[n] = t.T;
    A.out1[n] = t.qx;
    A.out2[n] = t.qy;
}

// non-equilibrium indicator, the 'B' parameter of Sec. 2.2 made
// dimensionless.  Isothermal sets: max over (2,0), (1,1), (0,2) of
// |a_km - rho ux^k uy^m| / rho.  Thermal sets: max of |P_ij - p delta_ij| / p
// (ij = xx, xy, yy) and |q_i| / (p sqrt(T)), p = rho T.
template <class ST, class SS, class OO>
__global__ void k_indicator(const NodeArgs A) {
    int i, j;
    if (!node_index(A.g, i, j)) return;
    int r = region_at(i, j, A.g);
    if (!(owns(r, A.self_high) || (!A.self_high && r == REG_IFACE))) return;
    using TB = typename SS::T;
    constexpr int N = SS::N;
    double f[SS::Q];
    load_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), f);
    if constexpr (SS::TH) {
        const ThermalState t = thermal_state<SS>(f);
        const double p = t.rho * t.T, pq = p * sqrt(t.T);
        double b = fabs(t.pxx - p) / p;
        b = fmax(b, fabs(t.pxy) / p);
        b = fmax(b, fabs(t.pyy - p) / p);
        b = fmax(b, fabs(t.qx) / pq);
        b = fmax(b, fabs(t.qy) / pq);
        A.out0[j * A.g.nx + i] = b;
        return;
    }
    double a00 = 0, a10 = 0, a01 = 0, a20 = 0, a11 = 0, a02 = 0;
#pragma unroll
    for (int a = 0; a < SS::Q; ++a) {
        double hx1 = TB::he.v[1][a % N], hy1 = TB::he.v[1][a / N];
        double hx2 = TB::he.v[2][a % N], hy2 = TB::he.v[2][a / N];
        a00 += f[a];
        a10 += f[a] * hx1;
        a01 += f[a] * hy1;
        a20 += f[a] * hx2;
        a11 += f[a] * hx1 * hy1;
        a02 += f[a] * hy2;
    }
    double rho = a00, ux = a10 / rho, uy = a01 / rho;
    double b = fabs(a20 - rho * ux * ux) / rho;
    b = fmax(b, fabs(a11 - rho * ux * uy) / rho);
    b = fmax(b, fabs(a02 - rho * uy * uy) / rho);
    A.out0[j * A.g.nx + i] = b;
}

// region change: nodes now in this set that were in the partner set get
// the projection of their partner-set populations (lift or restriction)
template <class ST, class SS, class OO>
__global__ void k_convert(const NodeArgs A) {
    if constexpr (OO::Q > 0) {
        int i, j;
        if (!node_index(A.g, i, j)) return;
        int r1 = region_at(i, j, A.g);
        if (!owns(r1, A.self_high)) return;
        int t = tile_of(i, A.g);
        int r0 = reg_of(A.oblo[t], A.obhi[t], j, A.g);
        if (!owns(r0, !A.self_high)) return;
        double fo[OO::Q], fs[SS::Q];
        load_node_d<ST, OO>(A.other, A.cur, i, j, sh_of(A), fo);
        const double *cl = nullptr;
        if (A.closure && A.self_high) cl = A.closure + (int64_t)(j * A.g.nx + i) * SS::Q;
        double cl36[SS::Q];
        if constexpr (OO::N == 3 && SS::N == 6 && !SS::TH) {
            // D2Q9 -> D2Q36 with the learned closure: the network's six
            // coefficients, zero elsewhere
            if (A.clw && A.self_high) {
                float c6[6];
                closure_coeffs<OO>(WBf16{A.clw}, A.cn, fo, A.ph.rho_ref, c6);
#pragma unroll
                for (int q = 0; q < SS::Q; ++q) cl36[q] = 0.0;
                cl36[3 * 6 + 0] = c6[0];
                cl36[0 * 6 + 3] = c6[1];
                cl36[3 * 6 + 1] = c6[2];
                cl36[1 * 6 + 3] = c6[3];
                cl36[4 * 6 + 0] = c6[4];
                cl36[0 * 6 + 4] = c6[5];
                cl = cl36;
            }
        }
        project_d<OO, SS>(fo, fs, cl);
        store_node_d<ST, SS>(A.self, A.cur, i, j, sh_of(A), fs);
    }
}

// Interface rows of the interpolation/extrapolation mode (Sec. 2.2): one
// thread per column and interface.  rho_I, u_I (and on thermal sets T_I) =
// averages of the low-side neighbour l and high-side neighbour h; in each
// set the population is the equilibrium at (rho_I, u_I, T_I) plus the
// same-side neighbour's non-equilibrium part.  The row beyond I on each side gets a copy of I in
// the other side's set (the second stencil row).  `recompute` = 0 keeps
// the stored I rows and only rebuilds copies and images.
template <class ST, class LS, class HS>
__global__ void k_paper_iface(const NodeArgs A, int copy, int recompute) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= 2 * A.g.nx) return;
    const int i = n % A.g.nx, top = n / A.g.nx;
    const int t = tile_of(i, A.g);
    const int lo = A.g.blo[t], hi = A.g.bhi[t];
    int jI, jl, jh;
    if (!top) {
        if (lo <= 0) return;
        jI = lo;
        jl = lo + 1;
        jh = lo - 1;
    } else {
        if (hi <= 0) return;
        jI = A.g.ny - hi;
        jl = jI - 1;
        jh = jI + 1;
    }
    const Buf &BL = A.self, &BH = A.other;
    double fL[LS::Q], fH[HS::Q];
    if (recompute) {
        double fl[LS::Q], fh[HS::Q], e1[HS::Q > LS::Q ? HS::Q : LS::Q], e2[HS::Q > LS::Q ? HS::Q : LS::Q];
        load_node_d<ST, LS>(BL, copy, i, jl, sh_of(A), fl);
        load_node_d<ST, HS>(BH, copy, i, jh, sh_of(A), fh);
        double rl, uxl, uyl, thl, rh, uxh, uyh, thh;
        moments_td<LS>(fl, rl, uxl, uyl, thl);
        moments_td<HS>(fh, rh, uxh, uyh, thh);
        double rI = 0.5 * (rl + rh), uxI = 0.5 * (uxl + uxh), uyI = 0.5 * (uyl + uyh);
        // T_I - 1 = ((T_l - 1) + (T_h - 1)) / 2
        double thI = 0.5 * (thl + thh);
        feq_d<LS>(rI, uxI, uyI, thI, e1);
        feq_d<LS>(rl, uxl, uyl, thl, e2);
#pragma unroll
        for (int a = 0; a < LS::Q; ++a) fL[a] = e1[a] + (fl[a] - e2[a]);
        feq_d<HS>(rI, uxI, uyI, thI, e1);
        feq_d<HS>(rh, uxh, uyh, thh, e2);
#pragma unroll
        for (int a = 0; a < HS::Q; ++a) fH[a] = e1[a] + (fh[a] - e2[a]);
    } else {
        load_node_d<ST, LS>(BL, copy, i, jI, sh_of(A), fL);
        load_node_d<ST, HS>(BH, copy, i, jI, sh_of(A), fH);
    }
    // I row in both sets, plus the copy beyond I on the opposite side
    emit_node<ST, LS>(BL, copy, i, jI, sh_of(A), fL, true, A.g, A.ph);
    emit_node<ST, LS>(BL, copy, i, jh, sh_of(A), fL, true, A.g, A.ph);
    emit_node<ST, HS>(BH, copy, i, jI, sh_of(A), fH, true, A.g, A.ph);
    emit_node<ST, HS>(BH, copy, i, jl, sh_of(A), fH, true, A.g, A.ph);
}

// Batched FP64 projection (test hook / closure training): n nodes, [node][Q]
template <class SS, class DD>
__global__ void k_project(const double *fs, const double *closure, double *fd, int64_t n) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double a[SS::Q], b[DD::Q];
#pragma unroll
    for (int q = 0; q < SS::Q; ++q) a[q] = fs[k * SS::Q + q];
    project_d<SS, DD>(a, b, closure ? closure + k * DD::Q : nullptr);
#pragma unroll
    for (int q = 0; q < DD::Q; ++q) fd[k * DD::Q + q] = b[q];
}

}  // namespace lbk

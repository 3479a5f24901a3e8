// lb_internal.hpp -- argument blocks shared by the host runtime and kernels.
//
// HBM layout of one velocity set: Q planes, one per population, each holding
// rows -2..ny+2 (two ghost rows beyond each wall) of `pitch` elements.
// Column c of row j of plane a lives at element
//     a * plane + rowbase + (j + 2) * pitch + c,      c in [-2, nx + 2)
// so the two left ghost columns of a row sit in the padding at the end of
// the previous row.  rowbase and pitch are multiples of 128 bytes, so every
// 64-column wave load of a row starts on a cache-line boundary.  Each set is
// allocated over the whole lattice; only the rows evolved in that set (plus
// two halo rows) are ever touched, so the extra capacity costs no traffic.
// Two copies (ping-pong) per set.
#pragma once
#include <stdint.h>

namespace lbi {

enum : int32_t { XBC_PERIODIC = 0, XBC_PRESSURE = 1 };
// YBC_SHEAR: a wall at the bottom, an imposed shear rate above the top row
enum : int32_t { YBC_WALLS = 0, YBC_PERIODIC = 1, YBC_SHEAR = 2 };
enum : int32_t { IF_HERMITE = 0, IF_PAPER = 1 };
enum : int32_t { TAU_CONST = 0, TAU_RHO = 1 };
enum : int32_t { REG_LOW = 0, REG_HIGH = 1, REG_IFACE = 2 };

struct Buf {
    char *base[2];     // ping-pong copies
    int64_t plane;     // elements per population plane
    int32_t pitch;     // elements per row
    int32_t rowbase;   // element offset of (row -2, column 0) in a plane
};

struct Geo {
    int32_t nx, ny, nrow, tile_w, ntiles, xbc, ybc, iface;
    const int32_t *blo;   // device: high rows at the bottom wall, per tile
    const int32_t *bhi;   // device: high rows at the top wall, per tile
};

struct Phys {
    double dt;         // time step
    double omega0;     // dt / tau at rho_ref
    double rho_ref;
    double rho_in, rho_out;
    double gx, gy;
    double uw[4];      // bottom x, y, top x, y
    double kn;         // Kn at rho_ref
    int32_t tau_mode;
    int32_t pad;
    double shear;      // YBC_SHEAR: velocity gradient du/dy imposed above the top row
};

// Storage shift: populations are stored as f - w_alpha s(i), with the
// reference density s(i) = s0 + ds * g(i) constant over each group
// g(i) = floor(i / SHIFT_GROUP) of SHIFT_GROUP columns -- the columns one
// work item of the update kernel owns, so that every node an item writes
// shares its shift.  ds = 0 except for pressure-driven lattices stored in
// FP32 / BF16, whose reference follows the imposed density ramp (the
// stored deviations then carry no density ramp); FP64 stores f (s = 0).
constexpr int SHIFT_GROUP = 60;
struct Shift {
    double s0, ds;
};

// Per-set kernel constants, in double and float: nu_p = x_p dt and
// k_p = |nu_p| (1 - |nu_p|) / 2 for the p-th 1D abscissa.
struct SetK {
    double nu[8], kk[8];
    float nuf[8], kkf[8];
    // diffuse walls [bottom, top]: S' = f_eq(1, u_wall, T_wall) - w per population,
    // K = sum_leaving |xi_y| w, D' = sum_leaving |xi_y| S'
    double sp[2][36], wK[2], wD[2];
    float spf[2][36], wKf[2], wDf[2];
};

// lifted nodes per wave of the closure inference kernel
constexpr int CLOSURE_NB = 16;

// Learned closure used by the lift (bf16 weights of the 10-64-64-8 network
// and the standardisation constants) -- see lb_mlp.hip
struct ClosureNorm {
    float xmean[10], xstd[10], tmean[6], tstd[6];
    float kn_ref;      // Kn at rho_ref (the input is log of the local Kn)
    int32_t tau_rho;   // local Kn ~ 1/rho
};

struct StepArgs {
    Geo g;
    Phys ph;
    Buf self, other;     // the set this kernel evolves, and its partner
    SetK ks;             // constants of `self`
    double rho_shift;    // storage shift s0 (Shift; rho_ref for F32/BF16, 0 for F64)
    double dshift;       // storage shift step per column group (Shift::ds)
    int32_t cur;         // source copy; the kernel writes copy cur ^ 1
    int32_t self_high;   // 1 if `self` is the high set
    int32_t nitems;      // work items (64 columns x a strip of rows)
    int32_t chunk;       // items per XCD slot (XCD-aware block mapping)
    const int32_t *items;   // device: 4 ints per item: i0, j0, j1, unused
    uint32_t seed;          // per-step seed of stochastic rounding (bf16 storage)
    float *clo;             // per lifted node: the 6 closure coefficients (NULL = analytic)
    const uint16_t *clw;    // closure weights (bf16)
    ClosureNorm cn;
};

// A batch of independent lattices stepped together: per-lattice arguments
// in device memory, one merged item list per kernel.
struct BatchArgs {
    const StepArgs *desc;   // device: per lattice, the StepArgs of this kernel's set
    const int32_t *items;   // device: 4 ints per item, the last names the lattice
    int32_t nitems;         // items (projection: entries projecting up)
    int32_t chunk;          // update: items per XCD slot
    int32_t cur;            // source copy of every lattice
    int32_t nsplit;         // projection: entries projecting down
    uint32_t seed;          // per-step seed of stochastic rounding (bf16 storage)
};

// One launch serving every velocity set (update) or every set pair
// (projection) of a batch: three slots of work items, each with its own item
// list, taking the blocks [start[s], start[s + 1]).  Update slots are the
// sets D2Q36, D2Q16, D2Q9; projection slots the pairs D2Q9/D2Q36,
// D2Q16/D2Q36, D2Q9/D2Q16.
// batch item of an 8-column periodic lattice (x neighbours wrapped inside
// 8-lane groups): its first entry is -(rows per group + NW_WRAP)
constexpr int32_t NW_WRAP = 0x10000;

struct BatchMulti {
    const StepArgs *desc;       // device: per lattice and side, as for BatchArgs
    const int32_t *items[3];    // device item lists (NULL for an empty slot)
    int32_t nitems[3];          // update: items; projection: entries projecting up
    int32_t nsplit[3];          // update: items per XCD slot; projection: entries projecting down
    int32_t start[4];           // first block of each slot; start[3] = blocks in the launch
    int32_t cur;                // source copy of every lattice
    uint32_t seed;              // per-step seed of stochastic rounding (bf16 storage)
};

// A persistent launch of a batch: `nsteps` steps of every lattice, each
// workgroup owning whole lattices (see k_batch_persistent).
struct PersistArgs {
    const StepArgs *desc;    // device: per lattice and side (low sides first), as for BatchMulti
    const int32_t *wl_off;   // per workgroup: its first entry of wl (grid + 1 entries)
    const int32_t *wl;       // lattice indices grouped by workgroup
    const int32_t *lat;      // per lattice, 8 ints: item offset, items, projection offset, up, down, pair, 0, 0
    const int32_t *items;    // update items (i0, j0, j1, descriptor index | set kind << 28)
    const int32_t *proj;     // projection entries (i, j, lattice, 0): a lattice's up entries, then its down ones
    int32_t nsteps;          // steps of this launch
    int32_t cur;             // source copy of the first step
    int64_t step0;           // step number of the first step (stochastic-rounding seeds)
};

// Arguments of the non-step kernels (one thread per node).
struct NodeArgs {
    Geo g;
    Phys ph;
    Buf self, other;
    double rho_shift;
    double dshift;
    int32_t cur;
    int32_t self_high;
    int32_t which;       // set index of `self` in the caller's numbering
    int32_t mode;        // kernel-specific variant (k_thermal: 1 = energy density)
    const double *in0, *in1, *in2;   // device FP64 inputs (fields or populations)
    const double *in3;               // device FP64 temperature field (thermal initialisation), or NULL
    double *out0, *out1, *out2;      // device FP64 outputs
    const int32_t *oblo, *obhi;      // previous bands (region change)
    const double *closure;           // optional closure coefficients (lift)
    const int32_t *nodes;            // node list (samples)
    int64_t nnodes;
    double theta;
    float *fx, *ft;                  // sample features / targets
    int32_t *flag;
    const uint16_t *clw;             // learned closure weights (bf16) for region-change lifts, or NULL
    ClosureNorm cn;
};

}  // namespace lbi

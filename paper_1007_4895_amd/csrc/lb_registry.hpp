// lb_registry.hpp -- table of compiled kernel instantiations.
//
// Each storage type has its own translation unit that instantiates the
// kernels for the (self set, partner set) pairs it supports and exposes them
// through one KernelSet per pair.  The host runtime looks pairs up here.
#pragma once
#include <hip/hip_runtime.h>

#include "lb_internal.hpp"

namespace lbk {

using StepFn = void (*)(const lbi::StepArgs &, int grid, hipStream_t);
using TimedFn = void (*)(const lbi::StepArgs &, int grid, hipStream_t, hipEvent_t start, hipEvent_t stop);
using NodeFn = void (*)(const lbi::NodeArgs &, int grid, hipStream_t);
using IfaceFn = void (*)(const lbi::NodeArgs &, int copy, int recompute, int grid, hipStream_t);
using ProjFn = void (*)(const double *, const double *, double *, int64_t, hipStream_t);
using BatchFn = void (*)(const lbi::BatchArgs &, int grid, hipStream_t);
// projection (nb_proj blocks) and finish pass over `fin` (nfin entries) in one launch
using ProjFinFn = void (*)(const lbi::StepArgs &, const int32_t *fin, int nfin, int nb_proj, int grid, hipStream_t);
// learned-closure steps: inference of the lifted nodes, the projection and
// the finish pass in one launch (nb_lift closure blocks, nb_down projection
// blocks, then the finish blocks up to grid)
using ProjClFn = void (*)(const lbi::StepArgs &, const int32_t *fin, int nfin, int nb_lift, int nb_down, int grid,
                          hipStream_t);
// both sets' updates in one launch (self = low set, D2Q9 only): the blocks
// of the high set come first
using PairFn = void (*)(const lbi::StepArgs &low, const lbi::StepArgs &high, int nb_high, int nb_low, hipStream_t,
                        hipEvent_t start, hipEvent_t stop);

struct KernelSet {
    int storage, nS, eqS, nO, eqO;
    int th;                 // thermal sets (temperature from each node's energy moment)
    StepFn update;
    TimedFn update_timed;   // the same launch bracketed by kernel start/stop events
    StepFn finish;        // valid when `self` is the low set of the pair
    StepFn project_halo;  // likewise
    ProjFinFn project_finish;   // likewise
    NodeFn refresh, init_eq, set_pop, get_pop, moments, indicator, convert;
    NodeFn thermal;         // temperature and heat flux (or energy density) per node
    IfaceFn paper_iface;   // valid when `self` is the low set of the pair
    ProjFn project;        // FP64 projection self -> partner
    StepFn closure_infer;   // learned-closure inference of the lifted nodes (self = low set)
    ProjClFn project_closure;   // closure + projection + finish in one launch; NULL but for D2Q9 / D2Q36
    NodeFn closure_samples; // training samples from an all-high run (self = high set)
    NodeFn closure_flags;   // the network's region flag into an indicator array (self = low set)
    PairFn update_pair;     // NULL unless the low set is D2Q9
    int pair_split;         // waves per block of update_pair (the high set's split)
    BatchFn finish_batch;   // batched forms (self = low set)
    BatchFn project_batch;
    const void *update_kernel;   // the __global__ symbol (for attribute queries)
};

// Kernels serving every velocity set (update) or set pair (projection) of a
// batch in one launch, for the sets D2Q36 of order eq6, D2Q16 of order eq4
// and D2Q9 (order 2).
using MultiFn = void (*)(const lbi::BatchMulti &, int grid, hipStream_t);
using PersistFn = void (*)(const lbi::PersistArgs &, int grid, hipStream_t);
struct MultiSet {
    int eq6, eq4;
    int waves;   // waves per block of the update (D2Q9 items per block)
    MultiFn update, project;
    PersistFn persist;   // the persistent launch (k_batch_persistent)
    int persist_waves;   // its waves per workgroup
};

struct Registry {
    const KernelSet *sets;
    int count;
    const MultiSet *multi;
    int nmulti;
};

// error reporting shared by the runtime's translation units
}  // namespace lbk
#include "../../include/lb.h"
lb_status lb_internal_fail(lb_status s, const char *msg);
namespace lbk {
void launch_to_bf16(const float *p, uint16_t *out, hipStream_t s);

Registry registry_f64();
Registry registry_f32();
Registry registry_bf16();
// thermal set pairs (FP64 and FP32 storage)
Registry registry_f64_thermal();
Registry registry_f32_thermal();

}  // namespace lbk

// lb_inst.hpp -- instantiation helpers for one storage type.
#pragma once
#include "lb_kernels.hpp"
#include "lb_registry.hpp"

#include <hip/hip_ext.h>

namespace lbk {

template <class ST, class S, class O>
struct Inst {
    static int nodes_grid(const NodeArgs &a) { return (a.g.nrow * a.g.nx + 255) / 256; }
    // FP32 / BF16 lattices whose storage reference varies by column group
    // take the kernels' XS variant
    static bool xs(const StepArgs &a) {
        if constexpr (sizeof(typename ST::M) == 4) return a.dshift != 0.0;
        else return false;
    }
    static void update(const StepArgs &a, int grid, hipStream_t s) {
        if constexpr (sizeof(typename ST::M) == 4) {
            if (xs(a)) {
                hipLaunchKernelGGL((k_update<ST, S, O, true>), dim3(grid), dim3(64 * update_split<S>()), 0, s, a);
                return;
            }
        }
        hipLaunchKernelGGL((k_update<ST, S, O>), dim3(grid), dim3(64 * update_split<S>()), 0, s, a);
    }
    static void update_timed(const StepArgs &a, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
        if constexpr (sizeof(typename ST::M) == 4) {
            if (xs(a)) {
                hipExtLaunchKernelGGL((k_update<ST, S, O, true>), dim3(grid), dim3(64 * update_split<S>()), 0, s, e0,
                                      e1, 0, a);
                return;
            }
        }
        hipExtLaunchKernelGGL((k_update<ST, S, O>), dim3(grid), dim3(64 * update_split<S>()), 0, s, e0, e1, 0, a);
    }
    static void finish(const StepArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_finish<ST, S, O>), dim3(grid), dim3(128), 0, s, a);
    }
    static void project_halo(const StepArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_project_halo<ST, S, O>), dim3(grid), dim3(128), 0, s, a);
    }
    static void project_finish(const StepArgs &a, const int32_t *fin, int nfin, int nbp, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_project_finish<ST, S, O>), dim3(grid), dim3(128), 0, s, a, fin, nfin, nbp);
    }
    static void project_closure(const StepArgs &a, const int32_t *fin, int nfin, int nbl, int nbd, int grid,
                                hipStream_t s) {
        hipLaunchKernelGGL((k_project_closure<ST, S, O>), dim3(grid), dim3(64), 0, s, a, fin, nfin, nbl, nbd);
    }
    static void closure_infer(const StepArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_closure_infer<ST, S, O>), dim3(grid), dim3(64), 0, s, a);
    }
    static void closure_flags(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_closure_flags<ST, S, O>), dim3(grid), dim3(64), 0, s, a);
    }
    static void closure_samples(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_closure_samples<ST, S, O>), dim3(grid), dim3(64), 0, s, a);
    }
    static void update_pair(const StepArgs &l, const StepArgs &h, int nb_h, int nb_l, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
        if constexpr (sizeof(typename ST::M) == 4) {
            if (xs(l)) {
                if (e0)
                    hipExtLaunchKernelGGL((k_update_pair<ST, S, O, true>), dim3(nb_h + nb_l), dim3(64 * pair_split<O>()),
                                          0, s, e0, e1, 0, l, h, nb_h);
                else
                    hipLaunchKernelGGL((k_update_pair<ST, S, O, true>), dim3(nb_h + nb_l), dim3(64 * pair_split<O>()),
                                       0, s, l, h, nb_h);
                return;
            }
        }
        if (e0)
            hipExtLaunchKernelGGL((k_update_pair<ST, S, O>), dim3(nb_h + nb_l), dim3(64 * pair_split<O>()), 0, s, e0,
                                  e1, 0, l, h, nb_h);
        else
            hipLaunchKernelGGL((k_update_pair<ST, S, O>), dim3(nb_h + nb_l), dim3(64 * pair_split<O>()), 0, s, l, h,
                               nb_h);
    }
    static void finish_batch(const BatchArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_finish_batch<ST, S, O>), dim3(grid), dim3(128), 0, s, a);
    }
    static void project_batch(const BatchArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_project_halo_batch<ST, S, O>), dim3(grid), dim3(128), 0, s, a);
    }
    static void refresh(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_refresh<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void init_eq(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_init_eq<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void set_pop(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_set_pop<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void get_pop(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_get_pop<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void moments(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_moments<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void indicator(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_indicator<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void thermal(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_thermal<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void convert(const NodeArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_convert<ST, S, O>), dim3(grid), dim3(256), 0, s, a);
    }
    static void paper_iface(const NodeArgs &a, int copy, int recompute, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_paper_iface<ST, S, O>), dim3(grid), dim3(256), 0, s, a, copy, recompute);
    }
    static void project(const double *fs, const double *cl, double *fd, int64_t n, hipStream_t s) {
        int grid = int((n + 127) / 128);
        if (grid > 0) hipLaunchKernelGGL((k_project<S, O>), dim3(grid), dim3(128), 0, s, fs, cl, fd, n);
    }
    static KernelSet make(int storage) {
        KernelSet k{};
        k.storage = storage;
        k.nS = S::N;
        k.eqS = S::EQ;
        k.nO = O::N;
        k.eqO = O::EQ;
        k.th = S::TH ? 1 : 0;
        k.update = &update;
        k.update_timed = &update_timed;
        k.finish = &finish;
        k.project_halo = &project_halo;
        k.project_finish = &project_finish;
        k.refresh = &refresh;
        k.init_eq = &init_eq;
        k.set_pop = &set_pop;
        k.get_pop = &get_pop;
        k.moments = &moments;
        k.indicator = &indicator;
        k.thermal = &thermal;
        k.convert = &convert;
        k.paper_iface = &paper_iface;
        k.project = &project;
        k.closure_infer = &closure_infer;
        k.project_closure = (S::N == 3 && O::N == 6 && !S::TH) ? &project_closure : nullptr;
        k.closure_samples = &closure_samples;
        k.closure_flags = &closure_flags;
        k.update_pair = update_split<S>() == 1 ? &update_pair : nullptr;
        k.pair_split = pair_split<O>();
        k.finish_batch = &finish_batch;
        k.project_batch = &project_batch;
        k.update_kernel = reinterpret_cast<const void *>(&k_update<ST, S, O>);
        return k;
    }
};

template <class ST, int E6, int E4>
struct MultiInst {
    static void update(const BatchMulti &m, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_update_multi<ST, lbt::VSet<6, E6>, lbt::VSet<4, E4>>), dim3(grid),
                           dim3(64 * multi_waves()), 0, s, m);
    }
    static void project(const BatchMulti &m, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_project_multi<ST, lbt::VSet<6, E6>, lbt::VSet<4, E4>>), dim3(grid), dim3(128), 0, s, m);
    }
    static void persist(const PersistArgs &a, int grid, hipStream_t s) {
        hipLaunchKernelGGL((k_batch_persistent<ST, lbt::VSet<6, E6>, lbt::VSet<4, E4>>), dim3(grid),
                           dim3(64 * PERSIST_WAVES), 0, s, a);
    }
    static MultiSet make() { return MultiSet{E6, E4, multi_waves(), &update, &project, &persist, PERSIST_WAVES}; }
};

}  // namespace lbk

#define LB_MULTI(ST, e6, e4) lbk::MultiInst<ST, e6, e4>::make()
#define LB_PAIR(ST, SID, n1, e1, n2, e2) \
    lbk::Inst<ST, lbt::VSet<n1, e1>, lbt::VSet<n2, e2>>::make(SID)
#define LB_PAIR_TH(ST, SID, n1, e1, n2, e2) \
    lbk::Inst<ST, lbt::VSet<n1, e1, true>, lbt::VSet<n2, e2, true>>::make(SID)

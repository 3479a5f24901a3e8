// Thermal lattices (temperature from each node's energy moment), FP64
// storage: the set pairs of the coupled channel and their uniform runs.
#include "lb_inst.hpp"

namespace lbk {
Registry registry_f64_thermal() {
    static const KernelSet sets[] = {
        LB_PAIR_TH(StF64, 0, 3, 2, 3, 2), LB_PAIR_TH(StF64, 0, 4, 3, 4, 3), LB_PAIR_TH(StF64, 0, 6, 4, 6, 4),
        LB_PAIR_TH(StF64, 0, 3, 2, 6, 4), LB_PAIR_TH(StF64, 0, 6, 4, 3, 2),
        LB_PAIR_TH(StF64, 0, 3, 2, 4, 3), LB_PAIR_TH(StF64, 0, 4, 3, 3, 2),
        LB_PAIR_TH(StF64, 0, 4, 3, 6, 4), LB_PAIR_TH(StF64, 0, 6, 4, 4, 3),
    };
    return Registry{sets, int(sizeof(sets) / sizeof(sets[0])), nullptr, 0};
}
}  // namespace lbk

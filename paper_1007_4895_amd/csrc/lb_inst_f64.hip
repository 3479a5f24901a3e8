// FP64 population storage: all supported set pairs (parity configurations).
#include "lb_inst.hpp"

namespace lbk {
Registry registry_f64() {
    static const KernelSet sets[] = {
        LB_PAIR(StF64, 0, 3, 2, 3, 2), LB_PAIR(StF64, 0, 4, 2, 4, 2), LB_PAIR(StF64, 0, 4, 3, 4, 3),
        LB_PAIR(StF64, 0, 6, 2, 6, 2), LB_PAIR(StF64, 0, 6, 4, 6, 4),
        LB_PAIR(StF64, 0, 3, 2, 4, 2), LB_PAIR(StF64, 0, 4, 2, 3, 2),
        LB_PAIR(StF64, 0, 3, 2, 4, 3), LB_PAIR(StF64, 0, 4, 3, 3, 2),
        LB_PAIR(StF64, 0, 3, 2, 6, 2), LB_PAIR(StF64, 0, 6, 2, 3, 2),
        LB_PAIR(StF64, 0, 3, 2, 6, 4), LB_PAIR(StF64, 0, 6, 4, 3, 2),
        LB_PAIR(StF64, 0, 4, 3, 6, 4), LB_PAIR(StF64, 0, 6, 4, 4, 3),
        LB_PAIR(StF64, 0, 4, 2, 6, 2), LB_PAIR(StF64, 0, 6, 2, 4, 2),
    };
    static const MultiSet multi[] = {LB_MULTI(StF64, 4, 3), LB_MULTI(StF64, 2, 2)};
    return Registry{sets, int(sizeof(sets) / sizeof(sets[0])), multi, int(sizeof(multi) / sizeof(multi[0]))};
}
}  // namespace lbk

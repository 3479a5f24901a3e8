// FP32 (weight-shifted) population storage.
#include "lb_inst.hpp"

namespace lbk {
Registry registry_f32() {
    static const KernelSet sets[] = {
        LB_PAIR(StF32, 1, 3, 2, 3, 2), LB_PAIR(StF32, 1, 4, 3, 4, 3), LB_PAIR(StF32, 1, 6, 4, 6, 4),
        LB_PAIR(StF32, 1, 3, 2, 6, 4), LB_PAIR(StF32, 1, 6, 4, 3, 2),
        LB_PAIR(StF32, 1, 3, 2, 4, 3), LB_PAIR(StF32, 1, 4, 3, 3, 2),
        LB_PAIR(StF32, 1, 4, 3, 6, 4), LB_PAIR(StF32, 1, 6, 4, 4, 3),
    };
    static const MultiSet multi[] = {LB_MULTI(StF32, 4, 3)};
    return Registry{sets, int(sizeof(sets) / sizeof(sets[0])), multi, int(sizeof(multi) / sizeof(multi[0]))};
}
}  // namespace lbk

// BF16 (weight-shifted) population storage, FP32 arithmetic.
#include "lb_inst.hpp"

namespace lbk {
Registry registry_bf16() {
    static const KernelSet sets[] = {
        LB_PAIR(StBF16, 2, 3, 2, 3, 2), LB_PAIR(StBF16, 2, 6, 4, 6, 4),
        LB_PAIR(StBF16, 2, 3, 2, 6, 4), LB_PAIR(StBF16, 2, 6, 4, 3, 2),
    };
    static const MultiSet multi[] = {LB_MULTI(StBF16, 4, 3)};
    return Registry{sets, int(sizeof(sets) / sizeof(sets[0])), multi, int(sizeof(multi) / sizeof(multi[0]))};
}
}  // namespace lbk

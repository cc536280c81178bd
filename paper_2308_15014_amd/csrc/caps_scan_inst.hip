// Instantiates the matrix-core scan kernels of one precision and kind
// (0 approximate keys, 1 exact main pass, 2 exact rescue pass, 3 exact main
// pass with survivor counts, 4 seed lists): compiled once
// per (CAPS_INST_PREC, CAPS_INST_KIND) pair so that they build in parallel.
#include "caps_mfma.h"

#if !defined(CAPS_INST_PREC) || !defined(CAPS_INST_KIND)
#error "compile with -DCAPS_INST_PREC=<CAPS_PREC_*> -DCAPS_INST_KIND=<0|1|2|3|4>"
#endif

namespace caps {

template <>
LowpFn pick_ns<CAPS_INST_PREC, CAPS_INST_KIND>(int ns, bool lab, int r) {
    constexpr int EX = CAPS_INST_KIND;
    switch (ns) {
        case 1: return pick_lab<CAPS_INST_PREC, 1, EX>(lab, r);
        case 2: return pick_lab<CAPS_INST_PREC, 2, EX>(lab, r);
        case 4: return pick_lab<CAPS_INST_PREC, 4, EX>(lab, r);
        default: return pick_lab<CAPS_INST_PREC, 8, EX>(lab, r);
    }
}

}  // namespace caps

// Instantiates the matrix-core scan kernels of one precision and key kind:
// compiled once per (CAPS_INST_PREC, CAPS_INST_EXACT) pair so that the
// instantiations build in parallel.
#include "caps_mfma.h"

#if !defined(CAPS_INST_PREC) || !defined(CAPS_INST_EXACT)
#error "compile with -DCAPS_INST_PREC=<CAPS_PREC_*> -DCAPS_INST_EXACT=<0|1>"
#endif

namespace caps {

template <>
LowpFn pick_ns<CAPS_INST_PREC, (bool)CAPS_INST_EXACT>(int ns, bool lab, int r) {
    constexpr bool EX = CAPS_INST_EXACT;
    switch (ns) {
        case 1: return pick_lab<CAPS_INST_PREC, 1, EX>(lab, r);
        case 2: return pick_lab<CAPS_INST_PREC, 2, EX>(lab, r);
        case 4: return pick_lab<CAPS_INST_PREC, 4, EX>(lab, r);
        default: return pick_lab<CAPS_INST_PREC, 8, EX>(lab, r);
    }
}

}  // namespace caps

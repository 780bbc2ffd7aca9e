// The M-specific launchers of the sweep kernels, for M = WLDA_KM.  The build
// compiles this file once per M (1..4), so the kernel variants of each M form
// a translation unit of their own.
#include "wlda_kernels_impl.h"

#ifndef WLDA_KM
#error "compile with -DWLDA_KM=<M>"
#endif

namespace wlda {

template <>
hipError_t seg_launch<WLDA_KM>(const PhaseArgs &a, uint32_t phase, const SegList &l, int bin, hipStream_t st) {
    if (phase == PH_WORD) return seg_dispatch<PH_WORD, WLDA_KM>(a, l, bin, st);
    return seg_dispatch<PH_DOC, WLDA_KM>(a, l, bin, st);
}

template <>
hipError_t long_launch<WLDA_KM>(const PhaseArgs &a, uint32_t phase, const LongList &l, hipStream_t st,
                                hipEvent_t *ev) {
    if (phase == PH_WORD) return long_dispatch<PH_WORD, WLDA_KM>(a, l, st, ev);
    return long_dispatch<PH_DOC, WLDA_KM>(a, l, st, ev);
}

template <>
hipError_t long_hist_launch<WLDA_KM>(const PhaseArgs &a, uint32_t phase, const LongList &l, hipStream_t st) {
    if (phase == PH_WORD) return long_hist_dispatch<PH_WORD, WLDA_KM>(a, l, st);
    return long_hist_dispatch<PH_DOC, WLDA_KM>(a, l, st);
}

}  // namespace wlda

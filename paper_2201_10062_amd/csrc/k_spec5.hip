// The fused sine-basis MINRES iteration instantiated for 5 time taps (BDF3 and BDF4, Sec. 4:
// the level t of (T y) combines y_t .. y_{t-4}); kept apart from k_spec.hip so that the two
// sets of instantiations compile in parallel.
#include "k_spec_impl.h"

namespace smr {

hipError_t run_one_taps5(hipStream_t st, const SpecP &P, int pprec, int cols, int mode, int blocks, int hp, int jph,
                         int pmode) {
  return run_one_taps<5>(st, P, pprec, cols, mode, blocks, hp, jph, pmode);
}

hipError_t run_multi_taps5(hipStream_t st, const SpecP *table, int ninst, int blocks, int hp, int cols, int pprec,
                           int mode, int jph, int pmode) {
  return run_multi_taps<5>(st, table, ninst, blocks, hp, cols, pprec, mode, jph, pmode);
}

}  // namespace smr

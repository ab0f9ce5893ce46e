// step_inst.hpp -- definitions and explicit instances of the step-kernel
// launchers for one storage precision, chosen by the including file through
// VANSE_S (storage type), VANSE_T (arithmetic type) and VANSE_SHIFT.
//
// Instances: workgroup widths 64, 128 and 256 for every feature variant the
// host selects (plain, force field, drag, both, a moving phi with both,
// solid nodes alone or with all of those, the scheme variants with all of
// those, FEAT_ALL), 512 for the plain
// step; the batched kernel for all but the last two (a moving phi is not
// batched); the two-step kernel of the first four, of solid nodes alone,
// with the drag, or with the force field and drag, of model B alone, with
// the drag, or with the force field and drag, of model B and of the Appendix
// B equilibrium, each with or without solid nodes, alone or with the force
// field and drag, and of a moving phi alone, with the drag, or
// with the force field and drag, with halves of step2_nt_of lanes, and its
// batched form (all but a moving phi) with halves of 64 lanes up to that
// width.
#include <type_traits>

#include "step_launch.hpp"

namespace vanse_dev {

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
void launch_step_nt(const StepGeom& g, const StepPhys<T>& ph, int blocks, hipStream_t st) {
  hipLaunchKernelGGL((vanse_step_kernel<S, T, SHIFT, WALLS, FEAT, NT>), dim3(blocks), dim3(NT), 0, st, g, ph);
}

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
void launch_step2(const StepGeom& g, const StepPhys<T>& ph, int blocks, hipStream_t st) {
  constexpr int NT = step2_nt_of(int(sizeof(T)), FEAT);
  static_assert(2 * step2_lds_bytes<S, T, FEAT, NT>() <= 160u * 1024u, "two workgroups per CU");
  hipLaunchKernelGGL((vanse_step2_kernel<S, T, SHIFT, WALLS, FEAT, NT>), dim3(blocks), dim3(2 * NT), 0,
                     st, g, ph);
}

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
bool launch_batch2(int threads, const BatchEntry<T>* entries, const int2* tile_map, int launch, int tiles,
                   hipStream_t st) {
  constexpr int MAXNT = step2_nt_of(int(sizeof(T)), FEAT);
  auto go = [&](auto nt) {
    constexpr int NT = decltype(nt)::value;
    hipLaunchKernelGGL((vanse_batch_step2_kernel<S, T, SHIFT, WALLS, FEAT, NT>), dim3(tiles), dim3(2 * NT),
                       0, st, entries, tile_map, launch);
  };
  if (threads == 64) {
    go(std::integral_constant<int, 64>{});
    return true;
  }
  if constexpr (MAXNT >= 128) {
    if (threads == 128) {
      go(std::integral_constant<int, 128>{});
      return true;
    }
  }
  if constexpr (MAXNT >= 256) {
    if (threads == 256) {
      go(std::integral_constant<int, 256>{});
      return true;
    }
  }
  return false;
}

template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
void launch_batch_nt(const BatchEntry<T>* entries, const int2* tile_map, int launch, int tiles,
                     hipStream_t st) {
  hipLaunchKernelGGL((vanse_batch_step_kernel<S, T, SHIFT, WALLS, FEAT, NT>), dim3(tiles), dim3(NT), 0,
                     st, entries, tile_map, launch);
}

#define VANSE_STEP_ONE(W, F, NT) \
  template void launch_step_nt<VANSE_S, VANSE_T, VANSE_SHIFT, W, F, NT>( \
      const StepGeom&, const StepPhys<VANSE_T>&, int, hipStream_t);
#define VANSE_BATCH_ONE(W, F, NT) \
  template void launch_batch_nt<VANSE_S, VANSE_T, VANSE_SHIFT, W, F, NT>( \
      const BatchEntry<VANSE_T>*, const int2*, int, int, hipStream_t);
#define VANSE_WIDTHS(M, W, F) M(W, F, 64) M(W, F, 128) M(W, F, 256)
#define VANSE_WALLS(M, F) VANSE_WIDTHS(M, false, F) VANSE_WIDTHS(M, true, F)

VANSE_WALLS(VANSE_STEP_ONE, 0)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_FORCE)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_MASK)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_MASK | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_MASK | FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_SCHEME | FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_STEP_ONE, FEAT_ALL)
VANSE_STEP_ONE(false, 0, 512)
VANSE_STEP_ONE(true, 0, 512)

VANSE_WALLS(VANSE_BATCH_ONE, 0)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_FORCE)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_DRAG)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_MASK)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_MASK | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_MASK | FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)
VANSE_WALLS(VANSE_BATCH_ONE, FEAT_SCHEME | FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)

// two steps per pass
#define VANSE_STEP2_ONE(W, F) \
  template void launch_step2<VANSE_S, VANSE_T, VANSE_SHIFT, W, F>( \
      const StepGeom&, const StepPhys<VANSE_T>&, int, hipStream_t); \
  template bool launch_batch2<VANSE_S, VANSE_T, VANSE_SHIFT, W, F>( \
      int, const BatchEntry<VANSE_T>*, const int2*, int, int, hipStream_t);
#define VANSE_STEP2_FEATS(W) VANSE_STEP2_ONE(W, 0) VANSE_STEP2_ONE(W, FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_FORCE) VANSE_STEP2_ONE(W, FEAT_FORCE | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_MASK) VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_FORCE | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_SCHEME) VANSE_STEP2_ONE(W, FEAT_SCHEME | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_EQ2) VANSE_STEP2_ONE(W, FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_SCHEME) VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_SCHEME | FEAT_FORCE | FEAT_DRAG) \
  VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_EQ2) VANSE_STEP2_ONE(W, FEAT_MASK | FEAT_EQ2 | FEAT_FORCE | FEAT_DRAG)
VANSE_STEP2_FEATS(false)
VANSE_STEP2_FEATS(true)
// a moving phi: one lattice at a time (not batched)
#define VANSE_STEP2_DYN(W, F) \
  template void launch_step2<VANSE_S, VANSE_T, VANSE_SHIFT, W, F>( \
      const StepGeom&, const StepPhys<VANSE_T>&, int, hipStream_t);
#define VANSE_STEP2_DYNS(W) VANSE_STEP2_DYN(W, FEAT_DYNPHI) VANSE_STEP2_DYN(W, FEAT_DYNPHI | FEAT_DRAG) \
  VANSE_STEP2_DYN(W, FEAT_DYNPHI | FEAT_FORCE | FEAT_DRAG)
VANSE_STEP2_DYNS(false)
VANSE_STEP2_DYNS(true)
#undef VANSE_STEP2_DYNS
#undef VANSE_STEP2_DYN
#undef VANSE_STEP2_FEATS
#undef VANSE_STEP2_ONE

#undef VANSE_STEP_ONE
#undef VANSE_BATCH_ONE
#undef VANSE_WIDTHS
#undef VANSE_WALLS

}  // namespace vanse_dev

// step_launch.hpp -- launchers of the step kernels.
//
// The kernel instances of each storage precision are compiled in a
// translation unit of their own (step_f64.hip, step_f32.hip, step_f32s.hip,
// step_f16s.hip, all built from step_inst.hpp) so that the library compiles
// in parallel; the host code only declares the launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "step2_kernel.hpp"
#include "step_kernel.hpp"

namespace vanse_dev {

// One lattice: `blocks` workgroups of NT lanes over the tiles of g.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
void launch_step_nt(const StepGeom& g, const StepPhys<T>& ph, int blocks, hipStream_t st);

// One lattice, two time steps per launch: `blocks` workgroups of two halves
// of step2_nt_of(sizeof(T), FEAT) lanes (FEAT: any of the force field, the
// drag and solid nodes).
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
void launch_step2(const StepGeom& g, const StepPhys<T>& ph, int blocks, hipStream_t st);

// Many lattices: one workgroup per tile of the batch table.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT, int NT>
void launch_batch_nt(const BatchEntry<T>* entries, const int2* tile_map, int launch, int tiles,
                     hipStream_t st);

// Many lattices, two time steps per launch: one workgroup of two halves of
// `threads` lanes (64, 128 or 256, at most step2_nt_of(sizeof(T), FEAT)) per
// tile of the batch table.  Returns false for a width not built.
template <typename S, typename T, bool SHIFT, bool WALLS, int FEAT>
bool launch_batch2(int threads, const BatchEntry<T>* entries, const int2* tile_map, int launch,
                   int tiles, hipStream_t st);

}  // namespace vanse_dev

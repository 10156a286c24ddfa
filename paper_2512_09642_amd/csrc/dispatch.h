// Declarations of the per-basis-width launchers.  Each is a template over the
// basis width S (and the basis precision T); its explicit instantiations for
// one S live in their own object, built from gram_s.hip with -DSSTEP_S=S, so
// the widths compile in parallel.  The dispatcher (kernels_fgs.hip) sees only
// these declarations.
#pragma once

#include "launch.h"

namespace sstep {

template <typename T, int S>
hipError_t gram_launch_s(const IterArgs &a, hipStream_t st);
template <typename T, int S>
hipError_t gram_op_launch_s(const IterArgs &a, hipStream_t st);
template <int S>
hipError_t fgs_launch_s(const IterArgs &a, hipStream_t st);
template <int S>
hipError_t fgs_rec_launch_s(const IterArgs &a, hipStream_t st);
template <int S>
hipError_t fgs_mom_launch_s(const IterArgs &a, hipStream_t st);
template <typename T, int S>
hipError_t gram_sym_launch_s(const IterArgs &a, hipStream_t st);
template <typename T, int S>
hipError_t bgram_launch_s(const BatchArgs &a, hipStream_t st);
template <int S>
hipError_t bfgs_launch_s(const BatchArgs &a, hipStream_t st);
template <typename T, int S>
hipError_t bgram_sym_launch_s(const BatchArgs &a, hipStream_t st);
template <int S>
hipError_t bfgs_rec_launch_s(const BatchArgs &a, hipStream_t st);
template <int S>
hipError_t bfgs_mom_launch_s(const BatchArgs &a, hipStream_t st);

}  // namespace sstep

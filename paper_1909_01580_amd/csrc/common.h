// Shared device helpers of the HGKS kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The per-lane arithmetic (reconstruction, flux) is also instantiated on the
// host by the operation-counting tool, hence host-and-device functions.
#define HGKS_FN __host__ __device__ __forceinline__

namespace hgks {

template <typename T> HGKS_FN T d_exp(T x);
template <> HGKS_FN double d_exp<double>(double x) { return exp(x); }
template <> HGKS_FN float d_exp<float>(float x) { return expf(x); }
template <typename T> HGKS_FN T d_erfc(T x);
template <> HGKS_FN double d_erfc<double>(double x) { return erfc(x); }
template <> HGKS_FN float d_erfc<float>(float x) { return erfcf(x); }
template <typename T> HGKS_FN T d_sqrt(T x);
template <> HGKS_FN double d_sqrt<double>(double x) { return sqrt(x); }
template <> HGKS_FN float d_sqrt<float>(float x) { return sqrtf(x); }
template <typename T> HGKS_FN T d_abs(T x) { return x < T(0) ? -x : x; }

// Workgroups are dispatched round-robin over the eight XCDs (block b runs
// on XCD b % 8).  Remapping gives every XCD one contiguous range of logical
// blocks, so that neighbouring tiles share an L2.  The grid must hold
// 8 * ceil(nb / 8) blocks; logical ids >= nb do nothing.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb_padded) {
  const unsigned per = nb_padded >> 3;
  return (b & 7u) * per + (b >> 3);
}

}  // namespace hgks

// dugks2p_fma.h -- internal interface between the library's runtime
// (dugks2p.hip) and the FMA-contracted build of the fused step
// (dugks2p_fma.hip).  Plain types only: the two translation units hold the
// same structs in different namespaces (dg, dg_fma), passed as bytes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

struct FmaStepArgs {
  const void *K;    // Consts
  size_t K_bytes;
  const void *w;    // Work
  size_t w_bytes;
  int fp32;         // 0: IoF64 state, 1: IoE32 state
  const void *src;  // IO policy of the current state
  const void *dst;  // IO policy of the next state
  size_t io_bytes;
  int sums_ready;   // phi and the f~ sums of src are already in w
  int shape;        // DUGKS2P_TILE_* (AUTO not allowed)
  int resident;     // the ping-pong state stays in the MALL (with_fused_kernel)
  hipStream_t stream;
  hipEvent_t e0, e1;  // optional: set to the tile kernel's start and end
};

// Enqueue one fused time step (cell macros and tile kernel, FMA-contracted
// arithmetic).  Returns hipSuccess or the first launch error; a size
// mismatch of the structs returns hipErrorInvalidValue.
hipError_t dugks2p_fma_step(const FmaStepArgs *a);

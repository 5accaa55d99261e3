// TEST INFRASTRUCTURE: the CPU emulation's form of the launch that records timing events (see
// hip_runtime.h): the start event, the launch, the stop event, in stream order.
#pragma once
#include "hip_runtime.h"
#define hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, e0, e1, flags, ...) \
  do {                                                                              \
    if (e0) hipEventRecord((e0), (stream));                                         \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);            \
    if (e1) hipEventRecord((e1), (stream));                                         \
  } while (0)

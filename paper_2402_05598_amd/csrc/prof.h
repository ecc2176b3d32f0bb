// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace fcgno {

// PK_LAYER: inner layers; PK_LAYER_FEAT / PK_LAYER_PROJ: the first (lift fused)
// and last (projection fused) layer kernels.
enum ProfKernel { PK_LAYER = 0, PK_SPECTRAL = 1, PK_DIR = 2, PK_WDOTS = 3, PK_UPDATE = 4, PK_ROWDFT = 5,
                  PK_TRAIN_FWD = 6, PK_TRAIN_BWD = 7, PK_LAYER_FEAT = 8, PK_LAYER_PROJ = 9, PK_COUNT = 10 };

bool prof_on();              // any family enabled
bool prof_on(int kernel);    // this family enabled
void prof_begin(int kernel, hipStream_t s);
void prof_end(int kernel, hipStream_t s);
// Accumulate the durations of completed event pairs (call after a stream sync).
void prof_collect();
// Event pair for a launch that carries its own events
// (hipExtLaunchKernelGGL).  False (no events) when the family is off.
bool prof_kernel_events(int kernel, hipEvent_t* start, hipEvent_t* stop);
void prof_kernel_done(int kernel, hipEvent_t start, hipEvent_t stop);

struct ProfScope {
  int k;
  hipStream_t s;
  ProfScope(int kernel, hipStream_t st) : k(kernel), s(st) { if (prof_on(k)) prof_begin(k, s); }
  ~ProfScope() { if (prof_on(k)) prof_end(k, s); }
};

}  // namespace fcgno

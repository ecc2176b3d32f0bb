// Optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

namespace fcgno {

enum ProfKernel { PK_LAYER = 0, PK_SPECTRAL = 1, PK_DIR = 2, PK_WDOTS = 3, PK_UPDATE = 4, PK_ROWDFT = 5,
                  PK_TRAIN_FWD = 6, PK_TRAIN_BWD = 7, PK_COUNT = 8 };

bool prof_on();
void prof_begin(int kernel, hipStream_t s);
void prof_end(int kernel, hipStream_t s);
// Accumulate the durations of completed event pairs (call after a stream sync).
void prof_collect();

struct ProfScope {
  int k;
  hipStream_t s;
  ProfScope(int kernel, hipStream_t st) : k(kernel), s(st) { if (prof_on()) prof_begin(k, s); }
  ~ProfScope() { if (prof_on()) prof_end(k, s); }
};

}  // namespace fcgno

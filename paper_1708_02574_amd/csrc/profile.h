// Kernel timing hooks used by the step-kernel launcher.
#pragma once

#include "tpa_internal.h"

namespace tpa {

// Record the start of a launch of variant `code` on `st`; returns a slot
// (or -1 when timing is off) to pass to profile_end after the launch.
int profile_begin(int code, hipStream_t st);
void profile_end(int slot, hipStream_t st);

}  // namespace tpa

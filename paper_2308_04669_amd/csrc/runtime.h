// Host runtime helpers shared by the C-ABI translation units.
#pragma once
#include <stdint.h>
#include <string>

namespace nedf {
void set_error(const std::string& msg);
int32_t fail(int32_t code, const std::string& msg);

// Kernel-level timing (nedf_profile_enable): when on, launches are bracketed
// by HIP events recorded on the launch stream under a stage name.
bool prof_on();
void prof_mark(const char* name, void* stream, bool begin);

// Tuning table (nedf_tune_*, nedf_autotune): chunks per superchunk of the
// matrix-core kernels, per kernel (NEDF_TUNE_*) and dtype.
int tune_value(int kernel, int dtype);
}  // namespace nedf

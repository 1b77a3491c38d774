// Optional per-kernel timing with HIP events recorded on the launching stream.
#pragma once

#include <hip/hip_runtime.h>

namespace rtn {

// Scope guard: records an event pair around the kernels launched inside it when
// profiling is enabled; does nothing otherwise.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();

 private:
  int slot_ = -1;
  hipStream_t st_ = nullptr;
};

bool profiling_on();

}  // namespace rtn

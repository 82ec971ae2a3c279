// profile.h -- scope that brackets a kernel launch with HIP events when
// SPGEMM_OPT_PROFILE is on (no cost otherwise beyond a flag test).
#pragma once
#include <hip/hip_runtime.h>

namespace mls {
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
  private:
    const char *name_;
    hipStream_t s_;
    hipEvent_t a_;
};
}  // namespace mls

#pragma once

#include "rans_internal.h"

namespace rans {

// RAII bracket of one kernel launch (no-op unless timing is enabled and
// `allowed`: callers that must not create events pass false).
class TimingScope {
public:
    TimingScope(int kind, hipStream_t st, bool allowed = true);
    ~TimingScope();
    TimingScope(const TimingScope&) = delete;
    TimingScope& operator=(const TimingScope&) = delete;

private:
    int kind_;
    hipStream_t st_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace rans

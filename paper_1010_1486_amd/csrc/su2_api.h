// su2_api.h -- exception barrier of the C ABI (host code only).
//
// No C++ exception may leave an extern "C" entry point: every entry point's
// body runs inside SU2_API_BEGIN / SU2_API_END (or SU2_API_END_SIZE for the
// size queries), which turn std::bad_alloc into SU2_ENOMEM and any other
// exception into SU2_EINVAL, each with a message for su2_last_error().
#pragma once

namespace su2rt {
int api_nomem() noexcept;
int api_unexpected() noexcept;
}  // namespace su2rt

#define SU2_API_BEGIN try {
#define SU2_API_END                                                                     \
    }                                                                                   \
    catch (const std::bad_alloc &) { return su2rt::api_nomem(); }                      \
    catch (...) { return su2rt::api_unexpected(); }
#define SU2_API_END_SIZE                                                                \
    }                                                                                   \
    catch (...) { return 0; }

// su2_api.h -- exception barrier and shared argument checks of the C ABI
// (host code only).
//
// No C++ exception may leave an extern "C" entry point: every entry point's
// body runs inside SU2_API_BEGIN / SU2_API_END (or SU2_API_END_SIZE for the
// size queries), which turn std::bad_alloc into SU2_ENOMEM and any other
// exception into SU2_EINVAL, each with a message for su2_last_error().
#pragma once

namespace su2rt {
int api_nomem() noexcept;
int api_unexpected() noexcept;

// The samplers draw a0 from sqrt(1 - a0^2) exp(alpha a0) with alpha = beta k
// >= 0 (their alpha < 1 branch accepts with probability exp(alpha (a0 - 1)),
// which is no probability for alpha < 0): beta must be finite and >= 0.
inline bool beta_ok(double beta) { return beta >= 0.0 && beta <= 1.7976931348623157e308; }
}  // namespace su2rt

#define SU2_API_BEGIN try {
#define SU2_API_END                                                                     \
    }                                                                                   \
    catch (const std::bad_alloc &) { return su2rt::api_nomem(); }                      \
    catch (...) { return su2rt::api_unexpected(); }
#define SU2_API_END_SIZE                                                                \
    }                                                                                   \
    catch (...) { return 0; }

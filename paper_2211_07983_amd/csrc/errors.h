// Error plumbing of the host engine: internal failures are C++ exceptions that
// the ABI boundary turns into an mps_status and a message on the context.
#pragma once

#include <string>

#include "../../include/mpsvqe.h"

struct Failure {
  mps_status code;
  std::string msg;
};

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess)                                                             \
      throw Failure{MPS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)};  \
  } while (0)

[[noreturn]] inline void fail(mps_status c, const std::string& m) { throw Failure{c, m}; }

// Error translation at the C boundary: no exception crosses an extern "C" function.
#pragma once

#include <new>

#include "internal.h"

#define DIFVM_API_BEGIN try {
#define DIFVM_API_END                                                    \
  }                                                                      \
  catch (const ::difvm::Error& e) {                                      \
    ::difvm::set_error(e.msg);                                           \
    return e.code;                                                       \
  }                                                                      \
  catch (const ::difvm::LayoutError& e) {                                \
    ::difvm::set_error(e.msg);                                           \
    return e.code;                                                       \
  }                                                                      \
  catch (const std::bad_alloc&) {                                        \
    ::difvm::set_error("host allocation failed");                        \
    return DIFVM_ERR_OOM;                                                \
  }                                                                      \
  catch (...) {                                                          \
    ::difvm::set_error("unexpected internal error");                     \
    return DIFVM_ERR_INVALID_ARG;                                        \
  }

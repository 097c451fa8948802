// Host stand-in for the HIP runtime header, so that the kernels' field code
// (paper_2402_09481_amd/csrc/field.h) compiles as plain C++ for the CPU checks
// of tests/test_field_host.py. Defines only what that header uses.
#pragma once
#include <stdint.h>
#define __device__
#define __host__
static inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }

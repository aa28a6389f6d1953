// Stand-in for the HIP runtime header when the register-DFT templates of
// csrc/cx.hpp are compiled for the host by tests/test_host_regdft.py: the
// qualifiers become plain C++ (the templates use no other HIP facility).
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline

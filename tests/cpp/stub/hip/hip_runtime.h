// Host stand-in for the HIP runtime header: lets the FFT headers of the
// library compile as plain C++ for the CPU checks of their transforms.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline

// Host stand-in for the HIP header, for tests/host/fft_check.cpp only: the
// line-transform header uses nothing of HIP but these qualifiers, so with
// them defined away its transforms compile for the CPU, where each lane is a
// thread and the exchange barrier a std::barrier.  Not part of the library.
#pragma once
#define __device__
#define __host__
#define __forceinline__ inline

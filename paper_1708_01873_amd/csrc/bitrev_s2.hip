// Kernels of libbitrev for 2-byte elements.
#define BITREV_S 2
#include "bitrev_kernels.inl"

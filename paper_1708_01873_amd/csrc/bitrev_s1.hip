// Kernels of libbitrev for 1-byte elements.
#define BITREV_S 1
#include "bitrev_kernels.inl"

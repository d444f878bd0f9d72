// Kernels of libbitrev for 4-byte elements.
#define BITREV_S 4
#include "bitrev_kernels.inl"

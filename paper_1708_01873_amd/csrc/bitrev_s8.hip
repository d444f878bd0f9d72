// Kernels of libbitrev for 8-byte elements.
#define BITREV_S 8
#include "bitrev_kernels.inl"

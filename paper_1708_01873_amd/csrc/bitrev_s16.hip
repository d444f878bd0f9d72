// Kernels of libbitrev for 16-byte elements.
#define BITREV_S 16
#include "bitrev_kernels.inl"

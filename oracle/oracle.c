/*
 * Bit-reversed permutation: the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library, and the GPU library
 * never calls it.
 *
 * Source: Knauth et al., "Practically efficient methods for performing
 * bit-reversed permutation in C++11 on the x86-64 architecture"
 * (arXiv:1708.01873).
 *
 * Definition followed (Introduction, and the listing that performs the
 * permutation with an external rev function): for n = 2^k elements, the
 * element at index i moves to index rev_k(i), where rev_k reverses exactly the
 * low k bits of i.  Because rev_k(rev_k(i)) = i, the permutation can be done in
 * place by swapping i with rev_k(i) once per pair, i.e. only when i < rev_k(i).
 *
 * Elements are opaque blocks of elem_size bytes: nothing is interpreted, so
 * NaN payloads and signed zeros move unchanged.  Parity with the GPU path is
 * byte-exact.
 *
 * Readings taken where the paper leaves a choice:
 *   - rev works on exactly k bits (the listing's rev is templated on the word
 *     size used for the reversal), not on a machine word;
 *   - k = 0 and k = 1 are the identity (the listing's loop is empty for N <= 2);
 *   - fixed points (i == rev_k(i)) never move;
 *   - batched offsets are counted in elements.
 *
 * Every function here is pinned by tests that do not use this file's
 * arithmetic: the paper's worked n = 8 example, the involution, an independent
 * byte-table reversal for every index up to k = 12, the inductive XOR
 * generator, the even-odd (Stockham) chain, the recursive square-transpose
 * decomposition and the swap-count closed form.
 */
#include <omp.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define ORACLE_MAX_LOG2N 62

/* Reverse the low k bits of i one bit at a time: Theta(k) per index, the
 * bitwise reversal the Introduction describes before the byte table. */
uint64_t oracle_rev(uint64_t i, int k)
{
    uint64_t r = 0;
    int j;
    for (j = 0; j < k; ++j)
        r = (r << 1) | ((i >> j) & 1u);
    return r;
}

static void swap_bytes(unsigned char *a, unsigned char *b, size_t s)
{
    size_t t;
    for (t = 0; t < s; ++t) {
        unsigned char tmp = a[t];
        a[t] = b[t];
        b[t] = tmp;
    }
}

/* In place, as in the Introduction's listing: visit every index, compute its
 * reversal and swap the pair once (only when index < reversed).  The first and
 * last index are their own reversals, so the listing's loop skips them; the
 * comparison handles them identically, so this loop visits all indices.
 * Returns 0, or -1 for an argument outside the domain. */
int oracle_inplace(void *data, int k, size_t elem_size)
{
    unsigned char *v = (unsigned char *)data;
    uint64_t n, i;
    if (k < 0 || k > ORACLE_MAX_LOG2N || elem_size == 0 || (data == NULL && k > 0))
        return -1;
    n = (uint64_t)1 << k;
    for (i = 0; i < n; ++i) {
        uint64_t r = oracle_rev(i, k);
        if (i < r)
            swap_bytes(v + i * elem_size, v + r * elem_size, elem_size);
    }
    return 0;
}

/* Out of place, the form Carter and Gatlin's buffered method writes
 * (Introduction, bit reversal using a matrix buffer): dest[rev(i)] <- src[i]
 * for every i.  src and dst must not overlap. */
int oracle_outofplace(const void *src, void *dst, int k, size_t elem_size)
{
    const unsigned char *in = (const unsigned char *)src;
    unsigned char *out = (unsigned char *)dst;
    uint64_t n, i;
    if (k < 0 || k > ORACLE_MAX_LOG2N || elem_size == 0 || src == NULL || dst == NULL)
        return -1;
    n = (uint64_t)1 << k;
    for (i = 0; i < n; ++i)
        memcpy(out + oracle_rev(i, k) * elem_size, in + i * elem_size, elem_size);
    return 0;
}

/* The same out-of-place definition with the index range split over the host
 * threads (OpenMP, static schedule): every i is still visited exactly once and
 * dest[rev(i)] <- src[i] with the bitwise rev above, so the result is
 * oracle_outofplace's.  It times the CPU baseline on all host cores and
 * computes the expected result of the multi-GiB comparisons, where the
 * one-thread loop would take minutes.  Returns the number of threads used, or
 * -1 for an argument outside the domain. */
int oracle_outofplace_mt(const void *src, void *dst, int k, size_t elem_size)
{
    const unsigned char *in = (const unsigned char *)src;
    unsigned char *out = (unsigned char *)dst;
    int64_t n;
    int threads = 1;
    if (k < 0 || k > ORACLE_MAX_LOG2N || elem_size == 0 || src == NULL || dst == NULL)
        return -1;
    n = (int64_t)1 << k;
#pragma omp parallel
    {
#pragma omp single
        threads = omp_get_num_threads();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            memcpy(out + oracle_rev((uint64_t)i, k) * elem_size, in + (uint64_t)i * elem_size,
                   elem_size);
    }
    return threads;
}

/* `rows` independent arrays of 2^k elements each, stored one after another.
 * src == dst means in place. */
int oracle_rows(const void *src, void *dst, int k, int64_t rows, size_t elem_size)
{
    int64_t r;
    size_t row_bytes;
    if (k < 0 || k > ORACLE_MAX_LOG2N || elem_size == 0 || rows < 0)
        return -1;
    row_bytes = ((size_t)1 << k) * elem_size;
    for (r = 0; r < rows; ++r) {
        const unsigned char *in = (const unsigned char *)src + (size_t)r * row_bytes;
        unsigned char *out = (unsigned char *)dst + (size_t)r * row_bytes;
        int rc = (src == dst) ? oracle_inplace(out, k, elem_size)
                              : oracle_outofplace(in, out, k, elem_size);
        if (rc != 0)
            return rc;
    }
    return 0;
}

/* Many arrays packed into one buffer: array a holds elements
 * [offsets[a], offsets[a+1]) and has 2^log2n[a] of them.  Each is permuted in
 * place independently.  Returns -1 (and stops) at the first array whose length
 * is not 2^log2n[a]. */
int oracle_batched(void *data, const int64_t *offsets, const int32_t *log2n,
                   int64_t num_arrays, size_t elem_size)
{
    int64_t a;
    if (num_arrays < 0 || elem_size == 0)
        return -1;
    for (a = 0; a < num_arrays; ++a) {
        int k = log2n[a];
        if (k < 0 || k > ORACLE_MAX_LOG2N)
            return -1;
        if (offsets[a + 1] - offsets[a] != ((int64_t)1 << k))
            return -1;
        if (oracle_inplace((unsigned char *)data + (size_t)offsets[a] * elem_size, k,
                           elem_size) != 0)
            return -1;
    }
    return 0;
}

/* Digit reversal for radix-2^d FFTs (the paper's Introduction motivates the
 * permutation by radix-2 decimation in time; a radix-2^d FFT splits by 2^d
 * residues at each level, and doing those splits up front reverses the order
 * of the base-2^d digits of each index).  k must be a multiple of d; the
 * digits are d-bit groups, least significant first, and their order is
 * reversed while each digit keeps its own bit order.  d = 1 is oracle_rev. */
uint64_t oracle_digit_rev(uint64_t i, int k, int d)
{
    uint64_t r = 0, mask;
    int j;
    if (d <= 0 || k % d)
        return ~(uint64_t)0;
    mask = ((uint64_t)1 << d) - 1;
    for (j = 0; j < k; j += d)
        r = (r << d) | ((i >> j) & mask);
    return r;
}

/* Out of place digit-reversed permutation: dst[drev(i)] <- src[i]. */
int oracle_digit_outofplace(const void *src, void *dst, int k, int d, size_t elem_size)
{
    const unsigned char *in = (const unsigned char *)src;
    unsigned char *out = (unsigned char *)dst;
    uint64_t n, i;
    if (k < 0 || k > ORACLE_MAX_LOG2N || d <= 0 || k % d || elem_size == 0 || !src || !dst)
        return -1;
    n = (uint64_t)1 << k;
    for (i = 0; i < n; ++i)
        memcpy(out + oracle_digit_rev(i, k, d) * elem_size, in + i * elem_size, elem_size);
    return 0;
}

/* In place: digit reversal is an involution too, so swap each pair once. */
int oracle_digit_inplace(void *data, int k, int d, size_t elem_size)
{
    unsigned char *v = (unsigned char *)data;
    uint64_t n, i;
    if (k < 0 || k > ORACLE_MAX_LOG2N || d <= 0 || k % d || elem_size == 0 || (!data && k > 0))
        return -1;
    n = (uint64_t)1 << k;
    for (i = 0; i < n; ++i) {
        uint64_t r = oracle_digit_rev(i, k, d);
        if (i < r)
            swap_bytes(v + i * elem_size, v + r * elem_size, elem_size);
    }
    return 0;
}

/* One even-odd split (Introduction, Stockham auto-sort): the even-indexed
 * elements go to the first half in order, the odd-indexed ones to the second
 * half -- the n/2 x 2 matrix transposition.  n = 2^k >= 2 out of place. */
int oracle_evenodd(const void *src, void *dst, int k, size_t elem_size)
{
    const unsigned char *in = (const unsigned char *)src;
    unsigned char *out = (unsigned char *)dst;
    uint64_t n, half, j;
    if (k < 1 || k > ORACLE_MAX_LOG2N || elem_size == 0 || !src || !dst)
        return -1;
    n = (uint64_t)1 << k;
    half = n / 2;
    for (j = 0; j < half; ++j) {
        memcpy(out + j * elem_size, in + (2 * j) * elem_size, elem_size);
        memcpy(out + (half + j) * elem_size, in + (2 * j + 1) * elem_size, elem_size);
    }
    return 0;
}

int oracle_version(void) { return 1; }

/* Oracle-side FP32 multiply-add chain (test infrastructure only).
 *
 * The plain FP32 comparison score of two unit signatures is defined as one
 * correctly rounded multiply-add per component, in ascending component order,
 * starting from +0.0f. C's fmaf is correctly rounded, so this file computes
 * that definition directly on the CPU. Built with -ffp-contract=off. */
#include <math.h>
#include <stdint.h>

float oracle_score32(const float* a, const float* b, int64_t k) {
    float acc = 0.0f;
    for (int64_t c = 0; c < k; ++c) acc = fmaf(a[c], b[c], acc);
    return acc;
}

void oracle_score32_pairs(const float* shat, int64_t k, const int64_t* i, const int64_t* j,
                          int64_t n, float* out) {
    for (int64_t p = 0; p < n; ++p) out[p] = oracle_score32(shat + i[p] * k, shat + j[p] * k, k);
}

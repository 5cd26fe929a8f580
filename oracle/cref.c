/*
 * Plain schoolbook ring arithmetic for the CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Products in Z_q[X]/(X^N + 1) (Sec. II.B): coefficient k of a*b is
 *   sum_{i+j=k} a_i b_j  -  sum_{i+j=k+N} a_i b_j   (mod q),
 * written out directly, O(N^2), with 128-bit accumulators.  Also the
 * definitional negacyclic transform (Sec. V): A_k = sum_j a_j psi^((2k+1) j).
 * No blocking, no transforms, no shared code with the GPU path.
 * Inputs are residues in [0, q) with q < 2^62.
 */
#include <stdint.h>

typedef unsigned __int128 u128;

/* Products a_i*b_j < 2^124; 16 of them fit in 128 bits, so reduce every 16 terms. */
static uint64_t coeff(const uint64_t *a, const uint64_t *b, int64_t n, int64_t k, uint64_t q) {
    u128 pos = 0, neg = 0;
    int cnt = 0;
    uint64_t pos_r = 0, neg_r = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t j = k - i;
        if (j >= 0) {
            pos += (u128)a[i] * b[j];
        } else {
            neg += (u128)a[i] * b[j + n];
        }
        if (++cnt == 16) {
            pos_r = (uint64_t)(((u128)pos_r + pos % q) % q);
            neg_r = (uint64_t)(((u128)neg_r + neg % q) % q);
            pos = neg = 0;
            cnt = 0;
        }
    }
    pos_r = (uint64_t)(((u128)pos_r + pos % q) % q);
    neg_r = (uint64_t)(((u128)neg_r + neg % q) % q);
    return pos_r >= neg_r ? pos_r - neg_r : pos_r + q - neg_r;
}

void oracle_negacyclic_mul(const uint64_t *a, const uint64_t *b, uint64_t *out, int64_t n, uint64_t q) {
    for (int64_t k = 0; k < n; k++) out[k] = coeff(a, b, n, k, q);
}

/* Only the coefficients listed in idx[0..m). */
void oracle_negacyclic_coeffs(const uint64_t *a, const uint64_t *b, const int64_t *idx, int64_t m,
                              uint64_t *out, int64_t n, uint64_t q) {
    for (int64_t r = 0; r < m; r++) out[r] = coeff(a, b, n, idx[r], q);
}

static uint64_t mulmod(uint64_t x, uint64_t y, uint64_t q) { return (uint64_t)(((u128)x * y) % q); }

/* A_k = sum_j a_j w_k^j with w_k = psi^(2k+1), by Horner's rule per k. */
void oracle_ntt_def(const uint64_t *a, uint64_t *out, int64_t n, uint64_t q, uint64_t psi) {
    uint64_t psi2 = mulmod(psi, psi, q), w = psi;
    for (int64_t k = 0; k < n; k++) {
        uint64_t acc = 0;
        for (int64_t j = n - 1; j >= 0; j--) {
            acc = mulmod(acc, w, q) + a[j];
            if (acc >= q) acc -= q;
        }
        out[k] = acc;
        w = mulmod(w, psi2, q);
    }
}

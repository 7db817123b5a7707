/*
 * Reference DES / Triple-DES (EDE) over independent 64-bit blocks (ECB).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it; the library never does, and the two share no
 * code, header, table or generator.
 *
 * It is deliberately plain and slow: every bit of key, text and intermediate
 * state is held in its own unsigned char, as in the paper's memory design
 * (Sec. IV-C), and every permutation is a 1-based gather exactly as the
 * paper's Appendix A tables print it.  No bit tricks, no tables derived from
 * the printed ones, no fusion across steps.
 *
 * Readings of points the paper leaves open (each is pinned by a test):
 *   - bit numbering: DES bit 1 is the most significant bit of byte 0, bytes
 *     in memory order, for keys, plaintext and ciphertext alike;
 *   - S-box addressing (Sec. III-B): row = 2*b1 + b6, column = b2b3b4b5,
 *     both 0-based; chunk s (1..8, left to right) uses box s; the 4-bit value
 *     is written most significant bit first;
 *   - the key-schedule rotations (Sec. III-A) are cumulative;
 *   - after round 16 the halves are combined as R16 || L16 before the final
 *     permutation (Sec. III-B), which is what makes decryption the same
 *     procedure with reversed round keys;
 *   - the key bundle is K1 || K2 || K3 (8 bytes each); parity bits
 *     (8, 16, ..., 64) are never read.
 *
 * The only parallelism is the paper's CPU baseline (Sec. V): an OpenMP
 * parallel-for over blocks.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- Appendix A constant arrays, transcribed as printed ---------------- */

/* Appendix A, permuted choice table (64 -> 56 bits) */
static const unsigned char pc_1[56] = {
    57, 49, 41, 33, 25, 17, 9,
    1,  58, 50, 42, 34, 26, 18,
    10, 2,  59, 51, 43, 35, 27,
    19, 11, 3,  60, 52, 44, 36,
    63, 55, 47, 39, 31, 23, 15,
    7,  62, 54, 46, 38, 30, 22,
    14, 6,  61, 53, 45, 37, 29,
    21, 13, 5,  28, 20, 12, 4};

/* Appendix A, per-round left-rotation amounts */
static const int shift_keys[16] = {1, 1, 2, 2, 2, 2, 2, 2,
                                   1, 2, 2, 2, 2, 2, 2, 1};

/* Appendix A, key-compression table (56 -> 48 bits) */
static const unsigned char pc_2[48] = {
    14, 17, 11, 24, 1,  5,
    3,  28, 15, 6,  21, 10,
    23, 19, 12, 4,  26, 8,
    16, 7,  27, 20, 13, 2,
    41, 52, 31, 37, 47, 55,
    30, 40, 51, 45, 33, 48,
    44, 49, 39, 56, 34, 53,
    46, 42, 50, 36, 29, 32};

/* Appendix A, initial permutation */
static const unsigned char initial_perm[64] = {
    58, 50, 42, 34, 26, 18, 10, 2,
    60, 52, 44, 36, 28, 20, 12, 4,
    62, 54, 46, 38, 30, 22, 14, 6,
    64, 56, 48, 40, 32, 24, 16, 8,
    57, 49, 41, 33, 25, 17, 9,  1,
    59, 51, 43, 35, 27, 19, 11, 3,
    61, 53, 45, 37, 29, 21, 13, 5,
    63, 55, 47, 39, 31, 23, 15, 7};

/* Appendix A, expansion D-box table (32 -> 48 bits) */
static const unsigned char exp_d[48] = {
    32, 1,  2,  3,  4,  5,  4,  5,
    6,  7,  8,  9,  8,  9,  10, 11,
    12, 13, 12, 13, 14, 15, 16, 17,
    16, 17, 18, 19, 20, 21, 20, 21,
    22, 23, 24, 25, 24, 25, 26, 27,
    28, 29, 28, 29, 30, 31, 32, 1};

/* Appendix A, the eight S-boxes, [box][row][column] */
static const unsigned char s_box[8][4][16] = {
    {{14, 4, 13, 1, 2, 15, 11, 8, 3, 10, 6, 12, 5, 9, 0, 7},
     {0, 15, 7, 4, 14, 2, 13, 1, 10, 6, 12, 11, 9, 5, 3, 8},
     {4, 1, 14, 8, 13, 6, 2, 11, 15, 12, 9, 7, 3, 10, 5, 0},
     {15, 12, 8, 2, 4, 9, 1, 7, 5, 11, 3, 14, 10, 0, 6, 13}},
    {{15, 1, 8, 14, 6, 11, 3, 4, 9, 7, 2, 13, 12, 0, 5, 10},
     {3, 13, 4, 7, 15, 2, 8, 14, 12, 0, 1, 10, 6, 9, 11, 5},
     {0, 14, 7, 11, 10, 4, 13, 1, 5, 8, 12, 6, 9, 3, 2, 15},
     {13, 8, 10, 1, 3, 15, 4, 2, 11, 6, 7, 12, 0, 5, 14, 9}},
    {{10, 0, 9, 14, 6, 3, 15, 5, 1, 13, 12, 7, 11, 4, 2, 8},
     {13, 7, 0, 9, 3, 4, 6, 10, 2, 8, 5, 14, 12, 11, 15, 1},
     {13, 6, 4, 9, 8, 15, 3, 0, 11, 1, 2, 12, 5, 10, 14, 7},
     {1, 10, 13, 0, 6, 9, 8, 7, 4, 15, 14, 3, 11, 5, 2, 12}},
    {{7, 13, 14, 3, 0, 6, 9, 10, 1, 2, 8, 5, 11, 12, 4, 15},
     {13, 8, 11, 5, 6, 15, 0, 3, 4, 7, 2, 12, 1, 10, 14, 9},
     {10, 6, 9, 0, 12, 11, 7, 13, 15, 1, 3, 14, 5, 2, 8, 4},
     {3, 15, 0, 6, 10, 1, 13, 8, 9, 4, 5, 11, 12, 7, 2, 14}},
    {{2, 12, 4, 1, 7, 10, 11, 6, 8, 5, 3, 15, 13, 0, 14, 9},
     {14, 11, 2, 12, 4, 7, 13, 1, 5, 0, 15, 10, 3, 9, 8, 6},
     {4, 2, 1, 11, 10, 13, 7, 8, 15, 9, 12, 5, 6, 3, 0, 14},
     {11, 8, 12, 7, 1, 14, 2, 13, 6, 15, 0, 9, 10, 4, 5, 3}},
    {{12, 1, 10, 15, 9, 2, 6, 8, 0, 13, 3, 4, 14, 7, 5, 11},
     {10, 15, 4, 2, 7, 12, 9, 5, 6, 1, 13, 14, 0, 11, 3, 8},
     {9, 14, 15, 5, 2, 8, 12, 3, 7, 0, 4, 10, 1, 13, 11, 6},
     {4, 3, 2, 12, 9, 5, 15, 10, 11, 14, 1, 7, 6, 0, 8, 13}},
    {{4, 11, 2, 14, 15, 0, 8, 13, 3, 12, 9, 7, 5, 10, 6, 1},
     {13, 0, 11, 7, 4, 9, 1, 10, 14, 3, 5, 12, 2, 15, 8, 6},
     {1, 4, 11, 13, 12, 3, 7, 14, 10, 15, 6, 8, 0, 5, 9, 2},
     {6, 11, 13, 8, 1, 4, 10, 7, 9, 5, 0, 15, 14, 2, 3, 12}},
    {{13, 2, 8, 4, 6, 15, 11, 1, 10, 9, 3, 14, 5, 0, 12, 7},
     {1, 15, 13, 8, 10, 3, 7, 4, 12, 5, 6, 11, 0, 14, 9, 2},
     {7, 11, 4, 1, 9, 12, 14, 2, 0, 6, 10, 13, 15, 3, 5, 8},
     {2, 1, 14, 7, 4, 10, 8, 13, 15, 12, 9, 0, 3, 5, 6, 11}}};

/* Appendix A, straight permutation table (32 -> 32 bits) */
static const unsigned char per[32] = {
    16, 7,  20, 21,
    29, 12, 28, 17,
    1,  15, 23, 26,
    5,  18, 31, 10,
    2,  8,  24, 14,
    32, 27, 3,  9,
    19, 13, 30, 6,
    22, 11, 4,  25};

/* Appendix A, final permutation */
static const unsigned char final_perm[64] = {
    40, 8, 48, 16, 56, 24, 64, 32,
    39, 7, 47, 15, 55, 23, 63, 31,
    38, 6, 46, 14, 54, 22, 62, 30,
    37, 5, 45, 13, 53, 21, 61, 29,
    36, 4, 44, 12, 52, 20, 60, 28,
    35, 3, 43, 11, 51, 19, 59, 27,
    34, 2, 42, 10, 50, 18, 58, 26,
    33, 1, 41, 9,  49, 17, 57, 25};

/* ---- bit-array helpers; every array below is 1-based (index 0 unused) -- */

/* Sec. III-A: "57th bit of the original key will be the 1st bit of the
 * permuted key", and the same rule for every table: out[j] = in[table[j]]. */
static void permute(unsigned char *out, const unsigned char *in,
                    const unsigned char *table, int n) {
    for (int j = 1; j <= n; j++) out[j] = in[table[j - 1]];
}

/* DES bit 8*i + j + 1 is bit (7 - j) of byte i. */
static void bytes_to_bits(const uint8_t *bytes, int nbytes, unsigned char *bits) {
    for (int i = 0; i < nbytes; i++)
        for (int j = 0; j < 8; j++) bits[8 * i + j + 1] = (bytes[i] >> (7 - j)) & 1;
}

static void bits_to_bytes(const unsigned char *bits, int nbytes, uint8_t *bytes) {
    for (int i = 0; i < nbytes; i++) {
        int v = 0;
        for (int j = 0; j < 8; j++) v = 2 * v + bits[8 * i + j + 1];
        bytes[i] = (uint8_t)v;
    }
}

/* Circular left shift of a 28-bit half, one position at a time. */
static void rotate_left_28(unsigned char *half, int positions) {
    for (int t = 0; t < positions; t++) {
        unsigned char first = half[1];
        for (int j = 1; j < 28; j++) half[j] = half[j + 1];
        half[28] = first;
    }
}

/* ---- Sec. III-A: key generation ---------------------------------------- */

typedef struct {
    unsigned char k[16][49]; /* round key i (0-based) in k[i][1..48] */
} round_keys;

static void key_schedule(const uint8_t key[8], round_keys *rk) {
    unsigned char kbits[65], cd[57], c[29], d[29], joined[57];
    bytes_to_bits(key, 8, kbits);
    permute(cd, kbits, pc_1, 56);                  /* 64 -> 56 bits     */
    for (int j = 1; j <= 28; j++) {                /* split in two 28s  */
        c[j] = cd[j];
        d[j] = cd[28 + j];
    }
    for (int i = 0; i < 16; i++) {                 /* 16 round keys     */
        rotate_left_28(c, shift_keys[i]);          /* cumulative shifts */
        rotate_left_28(d, shift_keys[i]);
        for (int j = 1; j <= 28; j++) {
            joined[j] = c[j];
            joined[28 + j] = d[j];
        }
        permute(rk->k[i], joined, pc_2, 48);       /* 56 -> 48 bits     */
    }
}

/* ---- Sec. III-B: encryption / decryption of one 64-bit block ----------- */

/* S-box step: row from the first and last bit, column from the middle four. */
static int sbox_value(int box, const unsigned char *six /* six[0..5] */) {
    int row = 2 * six[0] + six[5];
    int col = 8 * six[1] + 4 * six[2] + 2 * six[3] + six[4];
    return s_box[box][row][col];
}

/* One DES pass.  decrypt != 0 applies the round keys in reverse order,
 * which is the paper's definition of decryption. */
static void des_bits(const unsigned char *in, unsigned char *out,
                     const round_keys *rk, int decrypt) {
    unsigned char t[65], left[33], right[33], e[49], x[49];
    unsigned char sub[33], f[33], new_right[33], pre[65];

    permute(t, in, initial_perm, 64);
    for (int j = 1; j <= 32; j++) {
        left[j] = t[j];
        right[j] = t[32 + j];
    }
    for (int round = 0; round < 16; round++) {
        const unsigned char *k = rk->k[decrypt ? 15 - round : round];
        permute(e, right, exp_d, 48);              /* expansion 32 -> 48 */
        for (int j = 1; j <= 48; j++) x[j] = e[j] ^ k[j];
        for (int b = 0; b < 8; b++) {              /* 8 S-boxes, 6 -> 4  */
            int v = sbox_value(b, &x[6 * b + 1]);
            for (int q = 0; q < 4; q++) sub[4 * b + q + 1] = (v >> (3 - q)) & 1;
        }
        permute(f, sub, per, 32);                  /* straight P-box     */
        for (int j = 1; j <= 32; j++) new_right[j] = left[j] ^ f[j];
        for (int j = 1; j <= 32; j++) {            /* swap halves        */
            left[j] = right[j];
            right[j] = new_right[j];
        }
    }
    for (int j = 1; j <= 32; j++) {                /* combine R16 || L16 */
        pre[j] = right[j];
        pre[32 + j] = left[j];
    }
    permute(out, pre, final_perm, 64);
}

/* ---- exported entry points ---------------------------------------------- */

/* Round keys of one 64-bit key, packed for comparison: round key bit j
 * (1..48) is bit (48 - j) of out[i], i.e. bit 1 is the most significant of
 * the low 48 bits. */
void oracle_key_schedule(const uint8_t key[8], uint64_t out[16]) {
    round_keys rk;
    key_schedule(key, &rk);
    for (int i = 0; i < 16; i++) {
        uint64_t v = 0;
        for (int j = 1; j <= 48; j++) v = 2 * v + rk.k[i][j];
        out[i] = v;
    }
}

/* S-box step alone: six_bits holds b1..b6 with b1 as its bit 5. */
int oracle_sbox(int box, int six_bits) {
    unsigned char six[6];
    for (int q = 0; q < 6; q++) six[q] = (six_bits >> (5 - q)) & 1;
    return sbox_value(box, six);
}

/* Single DES, ECB, nbytes a multiple of 8 (anything past the last whole
 * block is left untouched). */
void oracle_des_ecb(const uint8_t key[8], const uint8_t *in, uint8_t *out,
                    size_t nbytes, int decrypt) {
    round_keys rk;
    key_schedule(key, &rk);
    long long nblocks = (long long)(nbytes / 8);
#pragma omp parallel for schedule(static)
    for (long long b = 0; b < nblocks; b++) {
        unsigned char p[65], c[65];
        bytes_to_bits(in + 8 * b, 8, p);
        des_bits(p, c, &rk, decrypt);
        bits_to_bytes(c, 8, out + 8 * b);
    }
}

/* Triple-DES EDE, ECB, on key bundle K1 || K2 || K3:
 *   encrypt: C = E_K3(D_K2(E_K1(P)))
 *   decrypt: P = D_K1(E_K2(D_K3(C)))   (Sec. III-B, the two 3DES equations) */
void oracle_tdes_ecb(const uint8_t key24[24], const uint8_t *in, uint8_t *out,
                     size_t nbytes, int decrypt) {
    round_keys rk1, rk2, rk3;
    key_schedule(key24, &rk1);
    key_schedule(key24 + 8, &rk2);
    key_schedule(key24 + 16, &rk3);
    long long nblocks = (long long)(nbytes / 8);
#pragma omp parallel for schedule(static)
    for (long long b = 0; b < nblocks; b++) {
        unsigned char a[65], c[65];
        bytes_to_bits(in + 8 * b, 8, a);
        if (!decrypt) {
            des_bits(a, c, &rk1, 0);
            des_bits(c, a, &rk2, 1);
            des_bits(a, c, &rk3, 0);
        } else {
            des_bits(a, c, &rk3, 1);
            des_bits(c, a, &rk2, 0);
            des_bits(a, c, &rk1, 1);
        }
        bits_to_bytes(c, 8, out + 8 * b);
    }
}

/* Copies of the transcribed tables, for the transcription checks.
 * which: 0 pc_1, 1 shift_keys, 2 pc_2, 3 initial_perm, 4 exp_d,
 *        5 s (8*4*16, box-major), 6 per, 7 final_perm.
 * Returns the number of entries written (at most cap), or -1. */
int oracle_table(int which, int *dst, int cap) {
    const unsigned char *src = NULL;
    int n = 0;
    switch (which) {
    case 0: src = pc_1; n = 56; break;
    case 1:
        for (int i = 0; i < 16 && i < cap; i++) dst[i] = shift_keys[i];
        return cap < 16 ? cap : 16;
    case 2: src = pc_2; n = 48; break;
    case 3: src = initial_perm; n = 64; break;
    case 4: src = exp_d; n = 48; break;
    case 5: src = &s_box[0][0][0]; n = 512; break;
    case 6: src = per; n = 32; break;
    case 7: src = final_perm; n = 64; break;
    default: return -1;
    }
    if (n > cap) n = cap;
    for (int i = 0; i < n; i++) dst[i] = src[i];
    return n;
}

int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

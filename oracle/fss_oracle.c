/*
 * fss_oracle.c -- plain, slow, obviously-correct CPU oracle for the masked-input
 * FSS hot path (DPF for equality predicates, DCF for range predicates).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  The product (the HIP
 * library under paper_2209_03526_amd/) never links, loads or calls it, and the
 * two share no code, header, table or constant generator.
 *
 * What it follows:
 *   - FSS scheme shape (Gen produces two keys, Eval(k_b, x) produces a share of
 *     f(x)): Def. 3, Sec. III-C.
 *   - DPF for point functions f^=_{alpha,beta}, DCF for comparison functions
 *     g^<_{alpha,beta}, interval containment built from DCFs, beta = 1 in Z_2:
 *     Sec. V-C (token generation), and the Z_2 output group of the token.
 *   - Masked-input evaluation (servers open x + r, keys are generated for the
 *     shifted function): Sec. V-C, the "basic approach" of Boyle et al.
 *   - Security parameter lambda = 128 (seeds and correction words are 128-bit
 *     AES blocks): Sec. VII-A, protocol instantiation.
 *   - AES-128 itself: FIPS-197 (Sec. 5.1 cipher, Sec. 5.2 key expansion).
 * The paper fixes neither the PRG nor the tree construction's bit conventions;
 * the readings taken here form this FSS specification
 * (PRG = fixed-key AES in Matyas-Meyer-Oseas form with the branch tweak XORed
 * into byte 0; tree walk MSB first; t = bit 0, v = bit 1, next seed = block with
 * bits 0 and 1 cleared; DPF and DCF both stop nu = n - 7 levels above the
 * leaves and end in a 128-bit leaf G_C(s) whose correction word answers the
 * last 7 input bits).
 * Share-level values (which random seed, which key bytes) therefore are pinned
 * only through AES and through the reconstruction identities; see the tests.
 *
 * Bit numbering of a 16-byte block: bit j is (byte[j >> 3] >> (j & 7)) & 1.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* AES-128 (FIPS-197), byte oriented, written from the standard.            */
/* ------------------------------------------------------------------------ */

static uint8_t g_sbox[256];

/* Multiplication in GF(2^8) modulo x^8 + x^4 + x^3 + x + 1 (FIPS-197 Sec. 4.2). */
static uint8_t gf_mul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    while (b) {
        if (b & 1) p ^= a;
        a = (uint8_t)((a << 1) ^ ((a & 0x80) ? 0x1b : 0x00));
        b >>= 1;
    }
    return p;
}

static uint8_t rotl8(uint8_t x, int k) { return (uint8_t)((x << k) | (x >> (8 - k))); }

/* S-box (FIPS-197 Sec. 5.1.1): multiplicative inverse in GF(2^8) (0 -> 0)
 * followed by the affine transformation b ^ rotl(b,1..4) ^ 0x63. */
__attribute__((constructor)) static void oracle_build_sbox(void)
{
    for (int x = 0; x < 256; x++) {
        uint8_t inv = 0;
        for (int y = 1; y < 256 && x != 0; y++)
            if (gf_mul((uint8_t)x, (uint8_t)y) == 1) { inv = (uint8_t)y; break; }
        g_sbox[x] = (uint8_t)(inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^ rotl8(inv, 3) ^
                              rotl8(inv, 4) ^ 0x63);
    }
}

uint8_t oracle_sbox(uint8_t x) { return g_sbox[x]; }

/* Key expansion (FIPS-197 Sec. 5.2): 44 words w[0..43], stored as 176 bytes. */
void oracle_aes128_expand(const uint8_t key[16], uint8_t rk[176])
{
    uint8_t rcon = 0x01;
    memcpy(rk, key, 16);
    for (int i = 4; i < 44; i++) {
        uint8_t temp[4];
        memcpy(temp, rk + 4 * (i - 1), 4);
        if (i % 4 == 0) {
            uint8_t t0 = temp[0];                 /* RotWord */
            temp[0] = temp[1]; temp[1] = temp[2]; temp[2] = temp[3]; temp[3] = t0;
            for (int k = 0; k < 4; k++) temp[k] = g_sbox[temp[k]];   /* SubWord */
            temp[0] ^= rcon;                      /* Rcon[i/4] = x^(i/4 - 1) */
            rcon = gf_mul(rcon, 0x02);
        }
        for (int k = 0; k < 4; k++) rk[4 * i + k] = (uint8_t)(rk[4 * (i - 4) + k] ^ temp[k]);
    }
}

/* Cipher (FIPS-197 Sec. 5.1).  state[r][c] = in[r + 4c]. */
void oracle_aes128_encrypt(const uint8_t rk[176], const uint8_t in[16], uint8_t out[16])
{
    uint8_t s[4][4];
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++) s[r][c] = in[r + 4 * c];

    for (int c = 0; c < 4; c++)                   /* AddRoundKey, round 0 */
        for (int r = 0; r < 4; r++) s[r][c] ^= rk[4 * c + r];

    for (int round = 1; round <= 10; round++) {
        for (int r = 0; r < 4; r++)               /* SubBytes */
            for (int c = 0; c < 4; c++) s[r][c] = g_sbox[s[r][c]];

        for (int r = 1; r < 4; r++) {             /* ShiftRows: row r rotates left by r */
            uint8_t t[4];
            for (int c = 0; c < 4; c++) t[c] = s[r][(c + r) % 4];
            for (int c = 0; c < 4; c++) s[r][c] = t[c];
        }

        if (round != 10) {                        /* MixColumns (Sec. 5.1.3) */
            for (int c = 0; c < 4; c++) {
                uint8_t a0 = s[0][c], a1 = s[1][c], a2 = s[2][c], a3 = s[3][c];
                s[0][c] = (uint8_t)(gf_mul(a0, 2) ^ gf_mul(a1, 3) ^ a2 ^ a3);
                s[1][c] = (uint8_t)(a0 ^ gf_mul(a1, 2) ^ gf_mul(a2, 3) ^ a3);
                s[2][c] = (uint8_t)(a0 ^ a1 ^ gf_mul(a2, 2) ^ gf_mul(a3, 3));
                s[3][c] = (uint8_t)(gf_mul(a0, 3) ^ a1 ^ a2 ^ gf_mul(a3, 2));
            }
        }

        for (int c = 0; c < 4; c++)               /* AddRoundKey */
            for (int r = 0; r < 4; r++) s[r][c] ^= rk[16 * round + 4 * c + r];
    }

    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++) out[r + 4 * c] = s[r][c];
}

/* ------------------------------------------------------------------------ */
/* Block helpers                                                             */
/* ------------------------------------------------------------------------ */

static int block_bit(const uint8_t b[16], int j) { return (b[j >> 3] >> (j & 7)) & 1; }

static void block_xor(uint8_t out[16], const uint8_t a[16], const uint8_t b[16])
{
    for (int k = 0; k < 16; k++) out[k] = (uint8_t)(a[k] ^ b[k]);
}

/* out = t ? out ^ cw : out */
static void block_xor_if(uint8_t out[16], int t, const uint8_t cw[16])
{
    if (t) for (int k = 0; k < 16; k++) out[k] ^= cw[k];
}

/* ------------------------------------------------------------------------ */
/* PRG: G_sigma(s) = AES_K(u) xor u with u = s xor sigma (sigma in byte 0),  */
/* fixed key K = 00 01 02 ... 0f.  sigma: 0 = left child, 1 = right child,   */
/* 2 = leaf/convert.                                                        */
/* ------------------------------------------------------------------------ */

static uint8_t g_prg_rk[176];
__attribute__((constructor(200))) static void oracle_build_prg_key(void)
{
    uint8_t k[16];
    oracle_build_sbox();
    for (int i = 0; i < 16; i++) k[i] = (uint8_t)i;
    oracle_aes128_expand(k, g_prg_rk);
}

void oracle_prg(int sigma, const uint8_t s[16], uint8_t out[16])
{
    uint8_t u[16], e[16];
    memcpy(u, s, 16);
    u[0] ^= (uint8_t)sigma;
    oracle_aes128_encrypt(g_prg_rk, u, e);
    block_xor(out, e, u);
}

/* Expansion of one seed into one child: (next seed with bits 0,1 cleared, t, v). */
static void expand(int sigma, const uint8_t s[16], uint8_t s_next[16], int *t, int *v)
{
    uint8_t w[16];
    oracle_prg(sigma, s, w);
    *t = block_bit(w, 0);
    *v = block_bit(w, 1);
    memcpy(s_next, w, 16);
    s_next[0] &= (uint8_t)~3u;
}

/* ------------------------------------------------------------------------ */
/* Counter-mode randomness of the simulated dealer:                          */
/*   K_seed = LE64(seed) || "OBLIVGM1"                                       */
/*   block  = AES_{K_seed}(LE16(domain) || LE16(j) || LE32(query) ||         */
/*                         LE32(pred) || LE32(elem))                          */
/* ------------------------------------------------------------------------ */

void oracle_rng_key(uint64_t seed, uint8_t rk[176])
{
    uint8_t k[16];
    for (int i = 0; i < 8; i++) k[i] = (uint8_t)(seed >> (8 * i));
    memcpy(k + 8, "OBLIVGM1", 8);
    oracle_aes128_expand(k, rk);
}

void oracle_rng_block_rk(const uint8_t rk[176], uint32_t domain, uint32_t j, uint32_t query,
                         uint32_t pred, uint32_t elem, uint8_t out[16])
{
    uint8_t in[16];
    in[0] = (uint8_t)domain; in[1] = (uint8_t)(domain >> 8);
    in[2] = (uint8_t)j;      in[3] = (uint8_t)(j >> 8);
    for (int i = 0; i < 4; i++) {
        in[4 + i]  = (uint8_t)(query >> (8 * i));
        in[8 + i]  = (uint8_t)(pred >> (8 * i));
        in[12 + i] = (uint8_t)(elem >> (8 * i));
    }
    oracle_aes128_encrypt(rk, in, out);
}

void oracle_rng_block(uint64_t seed, uint32_t domain, uint32_t j, uint32_t query, uint32_t pred,
                      uint32_t elem, uint8_t out[16])
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
    oracle_rng_block_rk(rk, domain, j, query, pred, elem, out);
}

/* ------------------------------------------------------------------------ */
/* Keys.                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint8_t  root[16];        /* s_b at the root */
    uint8_t  scw[32][16];     /* seed correction word of level i (i = 0..nu-1) */
    uint32_t tl, tr;          /* bit i: left / right t-correction bit of level i */
    uint8_t  cwout[16];       /* leaf correction word (128 outputs) */
} oracle_dpf_key;

typedef struct {
    uint8_t  root[16];
    uint8_t  scw[32][16];     /* level i = 0..nu-1, nu = n - 7 */
    uint32_t tl, tr, vcw;     /* bit i: t-left, t-right and value correction of level i;
                                 vcw bit 31: wrap share c_b (upper-bound half of a range key) */
    uint8_t  cwleaf[16];      /* leaf correction word: 128 outputs for the last 7 input bits */
} oracle_dcf_key;

typedef struct {
    oracle_dcf_key upper;     /* DCF at U = hi + r */
    oracle_dcf_key lower;     /* DCF at L = lo + r */
} oracle_range_key;

static uint32_t dom_mask(uint32_t n) { return n >= 32 ? 0xffffffffu : ((1u << n) - 1u); }

/* Bit i (1-based, MSB first) of an n-bit value, as in the tree walk: x_i. */
static int msb_bit(uint32_t x, uint32_t n, uint32_t i) { return (int)((x >> (n - i)) & 1u); }

/* DPF Gen for f^=_{alpha,1} over n-bit inputs (BGI tree with early termination
 * nu = n - 7 levels, leaf block carrying 128 output bits).  Roots s0, s1 have
 * bits 0,1 cleared; t0 = 0, t1 = 1. */
void oracle_dpf_gen(uint32_t n, uint32_t alpha, const uint8_t root0[16], const uint8_t root1[16],
                    oracle_dpf_key *k0, oracle_dpf_key *k1)
{
    uint32_t nu = n - 7;
    uint8_t s[2][16];
    int t[2] = {0, 1};
    memset(k0, 0, sizeof *k0);
    memset(k1, 0, sizeof *k1);
    memcpy(s[0], root0, 16);
    memcpy(s[1], root1, 16);
    memcpy(k0->root, root0, 16);
    memcpy(k1->root, root1, 16);

    for (uint32_t i = 1; i <= nu; i++) {
        uint8_t sl[2][16], sr[2][16];
        int tlb[2], trb[2], vdummy;
        for (int b = 0; b < 2; b++) {
            expand(0, s[b], sl[b], &tlb[b], &vdummy);
            expand(1, s[b], sr[b], &trb[b], &vdummy);
        }
        int a = msb_bit(alpha, n, i);
        /* keep the child on alpha's path, correct the other ("lose") one */
        uint8_t (*keep)[16] = a ? sr : sl;
        uint8_t (*lose)[16] = a ? sl : sr;
        int *tkeep = a ? trb : tlb;
        uint8_t scw[16];
        block_xor(scw, lose[0], lose[1]);
        int tlcw = tlb[0] ^ tlb[1] ^ a ^ 1;
        int trcw = trb[0] ^ trb[1] ^ a;
        int tkeepcw = a ? trcw : tlcw;

        for (int b = 0; b < 2; b++) {
            uint8_t ns[16];
            memcpy(ns, keep[b], 16);
            block_xor_if(ns, t[b], scw);
            int nt = tkeep[b] ^ (t[b] & tkeepcw);
            memcpy(s[b], ns, 16);
            t[b] = nt;
        }
        memcpy(k0->scw[i - 1], scw, 16);
        memcpy(k1->scw[i - 1], scw, 16);
        k0->tl |= (uint32_t)tlcw << (i - 1);
        k0->tr |= (uint32_t)trcw << (i - 1);
    }
    k1->tl = k0->tl;
    k1->tr = k0->tr;

    /* Leaf: CW_out = G_C(s_0) xor G_C(s_1) xor e_{alpha mod 128}. */
    uint8_t g0[16], g1[16], cw[16];
    oracle_prg(2, s[0], g0);
    oracle_prg(2, s[1], g1);
    block_xor(cw, g0, g1);
    uint32_t low = alpha & 127u;
    cw[low >> 3] ^= (uint8_t)(1u << (low & 7));
    memcpy(k0->cwout, cw, 16);
    memcpy(k1->cwout, cw, 16);
}

int oracle_dpf_eval(int party, const oracle_dpf_key *k, uint32_t n, uint32_t x)
{
    uint32_t nu = n - 7;
    uint8_t s[16];
    int t = party;
    x &= dom_mask(n);
    memcpy(s, k->root, 16);
    for (uint32_t i = 1; i <= nu; i++) {
        int xi = msb_bit(x, n, i);
        uint8_t ns[16];
        int nt, v;
        expand(xi, s, ns, &nt, &v);
        block_xor_if(ns, t, k->scw[i - 1]);
        int tcw = (int)(((xi ? k->tr : k->tl) >> (i - 1)) & 1u);
        nt ^= t & tcw;
        memcpy(s, ns, 16);
        t = nt;
    }
    uint8_t g[16];
    oracle_prg(2, s, g);
    block_xor_if(g, t, k->cwout);
    return block_bit(g, (int)(x & 127u));
}

/* DCF Gen for g^<_{alpha,1} over n-bit inputs with output in Z_2.  The tree
 * is walked for the nu = n - 7 high input bits; V_alpha accumulates the value
 * corrections along alpha's path.  The last 7 input bits are answered, as in
 * the DPF, by a 128-bit leaf G_C(s) corrected on alpha's path: once the
 * evaluation path has left alpha's path its two seeds and t bits are equal,
 * the leaves cancel and the value bits already hold [x < alpha]; on alpha's
 * path the leaf must reconstruct to [x_lo < alpha_lo] xor V_alpha. */
void oracle_dcf_gen(uint32_t n, uint32_t alpha, const uint8_t root0[16], const uint8_t root1[16],
                    oracle_dcf_key *k0, oracle_dcf_key *k1)
{
    uint32_t nu = n - 7;
    uint8_t s[2][16];
    int t[2] = {0, 1};
    int valpha = 0;
    memset(k0, 0, sizeof *k0);
    memset(k1, 0, sizeof *k1);
    memcpy(s[0], root0, 16);
    memcpy(s[1], root1, 16);
    memcpy(k0->root, root0, 16);
    memcpy(k1->root, root1, 16);

    for (uint32_t i = 1; i <= nu; i++) {
        uint8_t sl[2][16], sr[2][16];
        int tlb[2], trb[2], vlb[2], vrb[2];
        for (int b = 0; b < 2; b++) {
            expand(0, s[b], sl[b], &tlb[b], &vlb[b]);
            expand(1, s[b], sr[b], &trb[b], &vrb[b]);
        }
        int a = msb_bit(alpha, n, i);
        uint8_t (*keep)[16] = a ? sr : sl;
        uint8_t (*lose)[16] = a ? sl : sr;
        int *tkeep = a ? trb : tlb;
        int *vkeep = a ? vrb : vlb;
        int *vlose = a ? vlb : vrb;

        uint8_t scw[16];
        block_xor(scw, lose[0], lose[1]);
        /* Leaving alpha's path to the left at a level where alpha_i = 1 means
         * x < alpha: that branch must reconstruct to beta = 1. */
        int vcw = vlose[0] ^ vlose[1] ^ valpha ^ a;
        valpha = valpha ^ vkeep[0] ^ vkeep[1] ^ vcw;
        int tlcw = tlb[0] ^ tlb[1] ^ a ^ 1;
        int trcw = trb[0] ^ trb[1] ^ a;
        int tkeepcw = a ? trcw : tlcw;

        for (int b = 0; b < 2; b++) {
            uint8_t ns[16];
            memcpy(ns, keep[b], 16);
            block_xor_if(ns, t[b], scw);
            int nt = tkeep[b] ^ (t[b] & tkeepcw);
            memcpy(s[b], ns, 16);
            t[b] = nt;
        }
        memcpy(k0->scw[i - 1], scw, 16);
        memcpy(k1->scw[i - 1], scw, 16);
        k0->tl |= (uint32_t)tlcw << (i - 1);
        k0->tr |= (uint32_t)trcw << (i - 1);
        k0->vcw |= (uint32_t)vcw << (i - 1);
    }
    /* Leaf: bit j of CW = bit j of G_C(s_0) xor G_C(s_1), xor [j < alpha mod 128],
     * xor V_alpha. */
    uint8_t g0[16], g1[16], cw[16];
    oracle_prg(2, s[0], g0);
    oracle_prg(2, s[1], g1);
    block_xor(cw, g0, g1);
    uint32_t low = alpha & 127u;
    for (uint32_t j = 0; j < 128; j++)
        if ((int)(j < low) ^ valpha) cw[j >> 3] ^= (uint8_t)(1u << (j & 7));
    memcpy(k0->cwleaf, cw, 16);
    memcpy(k1->cwleaf, cw, 16);
    k1->tl = k0->tl;
    k1->tr = k0->tr;
    k1->vcw = k0->vcw;
}

int oracle_dcf_eval(int party, const oracle_dcf_key *k, uint32_t n, uint32_t x)
{
    uint32_t nu = n - 7;
    uint8_t s[16];
    int t = party;
    int v = 0;
    x &= dom_mask(n);
    memcpy(s, k->root, 16);
    for (uint32_t i = 1; i <= nu; i++) {
        int xi = msb_bit(x, n, i);
        uint8_t ns[16];
        int nt, nv;
        expand(xi, s, ns, &nt, &nv);
        v ^= nv ^ (t & (int)((k->vcw >> (i - 1)) & 1u));
        block_xor_if(ns, t, k->scw[i - 1]);
        int tcw = (int)(((xi ? k->tr : k->tl) >> (i - 1)) & 1u);
        nt ^= t & tcw;
        memcpy(s, ns, 16);
        t = nt;
    }
    uint8_t g[16];
    oracle_prg(2, s, g);
    block_xor_if(g, t, k->cwleaf);
    return v ^ block_bit(g, (int)(x & 127u));
}

/* ------------------------------------------------------------------------ */
/* Dealer: masked-input keys for one predicate over a column of rows.        */
/* RNG domain 3 ("FSS root seeds"): j = 0,1 roots of the DPF / of the upper  */
/* DCF, j = 2 wrap-share c_0 (bit 0), j = 3,4 roots of the lower DCF.        */
/* ------------------------------------------------------------------------ */

static void root_seed(const uint8_t rk[176], uint32_t j, uint32_t query, uint32_t pred,
                      uint32_t elem, uint8_t out[16])
{
    oracle_rng_block_rk(rk, 3, j, query, pred, elem, out);
    out[0] &= (uint8_t)~3u;
}

/* Equality predicate x == a: DPF at alpha = a + r (mod 2^n). */
/* Row e of the output is the key of table row rows[e] (rows == NULL: row e);
 * r[e] is that row's mask. */
void oracle_keygen_eq(uint32_t n, uint64_t seed, uint32_t query, uint32_t pred, uint32_t a,
                      const uint32_t *r, const uint32_t *rows, size_t count, oracle_dpf_key *k0,
                      oracle_dpf_key *k1)
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++) {
        uint8_t r0[16], r1[16];
        uint32_t row = rows ? rows[e] : (uint32_t)e;
        root_seed(rk, 0, query, pred, row, r0);
        root_seed(rk, 1, query, pred, row, r1);
        uint32_t alpha = (a + r[e]) & dom_mask(n);
        oracle_dpf_gen(n, alpha, r0, r1, &k0[e], &k1[e]);
    }
}

/* Range predicate lo <= x < hi: with L = lo + r and U = hi + r (mod 2^n),
 * [lo <= x < hi] = [xhat < U] xor [xhat < L] xor [L > U].  The public-to-the-
 * dealer bit [L > U] is split as c_0 (random) and c_1 = c_0 xor [L > U]. */
void oracle_keygen_range(uint32_t n, uint64_t seed, uint32_t query, uint32_t pred, uint32_t lo,
                         uint32_t hi, const uint32_t *r, const uint32_t *rows, size_t count,
                         oracle_range_key *k0, oracle_range_key *k1)
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++) {
        uint8_t u0[16], u1[16], l0[16], l1[16], cb[16];
        uint32_t row = rows ? rows[e] : (uint32_t)e;
        root_seed(rk, 0, query, pred, row, u0);
        root_seed(rk, 1, query, pred, row, u1);
        root_seed(rk, 3, query, pred, row, l0);
        root_seed(rk, 4, query, pred, row, l1);
        oracle_rng_block_rk(rk, 3, 2, query, pred, row, cb);
        uint32_t L = (lo + r[e]) & dom_mask(n);
        uint32_t U = (hi + r[e]) & dom_mask(n);
        oracle_dcf_gen(n, U, u0, u1, &k0[e].upper, &k1[e].upper);
        oracle_dcf_gen(n, L, l0, l1, &k0[e].lower, &k1[e].lower);
        uint32_t c0 = (uint32_t)block_bit(cb, 0);
        uint32_t c1 = c0 ^ (L > U ? 1u : 0u);
        k0[e].upper.vcw |= c0 << 31;
        k1[e].upper.vcw |= c1 << 31;
    }
}

/* Party b's share bit for each row; out[e] in {0,1}. */
void oracle_eval_eq(uint32_t n, int party, const oracle_dpf_key *k, const uint32_t *xhat,
                    size_t count, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++)
        out[e] = (uint8_t)oracle_dpf_eval(party, &k[e], n, xhat[e]);
}

void oracle_eval_range(uint32_t n, int party, const oracle_range_key *k, const uint32_t *xhat,
                       size_t count, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++) {
        int yu = oracle_dcf_eval(party, &k[e].upper, n, xhat[e]);
        int yl = oracle_dcf_eval(party, &k[e].lower, n, xhat[e]);
        int c = (int)(k[e].upper.vcw >> 31);
        out[e] = (uint8_t)(yu ^ yl ^ c);
    }
}

/* Single-key entry points for the pins (unmasked DPF/DCF of any alpha). */
void oracle_dpf_gen_seeded(uint32_t n, uint32_t alpha, uint64_t seed, uint32_t elem,
                           oracle_dpf_key *k0, oracle_dpf_key *k1)
{
    uint8_t rk[176], r0[16], r1[16];
    oracle_rng_key(seed, rk);
    root_seed(rk, 0, 0, 0, elem, r0);
    root_seed(rk, 1, 0, 0, elem, r1);
    oracle_dpf_gen(n, alpha, r0, r1, k0, k1);
}

void oracle_dcf_gen_seeded(uint32_t n, uint32_t alpha, uint64_t seed, uint32_t elem,
                           oracle_dcf_key *k0, oracle_dcf_key *k1)
{
    uint8_t rk[176], r0[16], r1[16];
    oracle_rng_key(seed, rk);
    root_seed(rk, 0, 0, 0, elem, r0);
    root_seed(rk, 1, 0, 0, elem, r1);
    oracle_dcf_gen(n, alpha, r0, r1, k0, k1);
}

/* Evaluate one key at many points (for exhaustive domain sweeps). */
void oracle_dpf_eval_points(int party, const oracle_dpf_key *k, uint32_t n, const uint32_t *x,
                            size_t count, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++) out[e] = (uint8_t)oracle_dpf_eval(party, k, n, x[e]);
}

void oracle_dcf_eval_points(int party, const oracle_dcf_key *k, uint32_t n, const uint32_t *x,
                            size_t count, uint8_t *out)
{
#pragma omp parallel for schedule(static)
    for (long long e = 0; e < (long long)count; e++) out[e] = (uint8_t)oracle_dcf_eval(party, k, n, x[e]);
}

/* ------------------------------------------------------------------------ */
/* Beaver triples for AND on packed words (RNG domain 4).  Random word k of  */
/* the stream for (query, and_id) is 32-bit word (k mod 4), little endian,   */
/* of block (domain 4, j = 0, query, and_id, elem = k / 4).  Triple word w   */
/* takes stream words 5w .. 5w+4 as a_0, a_1, b_0, b_1, c_0, and            */
/* c_1 = (a_0 ^ a_1) & (b_0 ^ b_1) ^ c_0.                                    */
/* ------------------------------------------------------------------------ */

static uint32_t le32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

/* Output slot i holds triple word words[i] (words == NULL: word i). */
void oracle_triples(uint64_t seed, uint32_t query, uint32_t and_id, const uint32_t *words,
                    size_t nwords, uint32_t *a0, uint32_t *a1, uint32_t *b0, uint32_t *b1,
                    uint32_t *c0, uint32_t *c1)
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
#pragma omp parallel for schedule(static)
    for (long long w = 0; w < (long long)nwords; w++) {
        uint32_t word[5];
        uint64_t wi = words ? words[w] : (uint64_t)w;
        for (int q = 0; q < 5; q++) {
            uint64_t k = 5ull * wi + (uint64_t)q;
            uint8_t blk[16];
            oracle_rng_block_rk(rk, 4, 0, query, and_id, (uint32_t)(k / 4), blk);
            word[q] = le32(blk + 4 * (k % 4));
        }
        a0[w] = word[0];
        a1[w] = word[1];
        b0[w] = word[2];
        b1[w] = word[3];
        c0[w] = word[4];
        c1[w] = ((word[0] ^ word[1]) & (word[2] ^ word[3])) ^ word[4];
    }
}

/* Dealer masks (RNG domain 2): r[i] = little-endian word 0 of block
 * (2, 0, query, pred, row_offset + i). */
void oracle_masks(uint64_t seed, uint32_t query, uint32_t pred, uint32_t row_offset, size_t count, uint32_t *r)
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)count; i++) {
        uint8_t blk[16];
        oracle_rng_block_rk(rk, 2, 0, query, pred, row_offset + (uint32_t)i, blk);
        r[i] = le32(blk);
    }
}

/* Consecutive counter blocks: out[16*i ..] = block (domain, j, query, pred,
 * elem0 + i) under K_seed, i = 0 .. count-1 (the same blocks as
 * oracle_rng_block, one key schedule for all of them). */
void oracle_rng_blocks(uint64_t seed, uint32_t domain, uint32_t j, uint32_t query, uint32_t pred, uint32_t elem0,
                       size_t count, uint8_t *out)
{
    uint8_t rk[176];
    oracle_rng_key(seed, rk);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)count; i++)
        oracle_rng_block_rk(rk, domain, j, query, pred, elem0 + (uint32_t)i, out + 16 * i);
}

size_t oracle_sizeof_dpf_key(void) { return sizeof(oracle_dpf_key); }
size_t oracle_sizeof_dcf_key(void) { return sizeof(oracle_dcf_key); }
size_t oracle_sizeof_range_key(void) { return sizeof(oracle_range_key); }

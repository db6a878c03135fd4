/* The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer: random
 * pattern sets and texts, brute force against Aho-Corasick at several chunk sizes and
 * thread counts, everything freed. Exit status 0 when every result agrees. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_brute(const uint8_t *pd, const uint64_t *po, uint32_t np, const uint8_t *text, uint64_t n, int threads,
              uint64_t **out, uint64_t *count);
void *orc_ac_build(const uint8_t *pd, const uint64_t *po, uint32_t np);
void orc_ac_free(void *h);
int orc_ac_scan(void *h, const uint8_t *text, uint64_t n, uint32_t alphabet, uint64_t chunk, int threads,
                uint64_t **out, uint64_t *count);
void orc_free(void *p);

static uint64_t st = 88172645463325252ull;
static uint32_t rnd(uint32_t n) {
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (uint32_t)(st % n);
}

int main(void) {
    int bad = 0;
    const uint32_t alphabets[] = {2, 4, 256};
    for (int t = 0; t < 200; t++) {
        const uint32_t a = alphabets[t % 3], np = 1 + rnd(30);
        uint64_t *po = (uint64_t *)malloc((np + 1) * sizeof(uint64_t));
        uint8_t *pd = (uint8_t *)malloc(np * 8 + 1);
        po[0] = 0;
        for (uint32_t j = 0; j < np; j++) {
            const uint32_t len = 1 + rnd(8);
            for (uint32_t i = 0; i < len; i++) pd[po[j] + i] = (uint8_t)rnd(a);
            po[j + 1] = po[j] + len;
        }
        const uint64_t n = rnd(700);
        uint8_t *text = (uint8_t *)malloc(n + 1);
        for (uint64_t i = 0; i < n; i++) text[i] = (uint8_t)rnd(a < 256 ? a + 1 : 256);
        uint64_t *kb = NULL, cb = 0;
        if (orc_brute(pd, po, np, text, n, 1 + (t % 4), &kb, &cb)) bad++;
        void *h = orc_ac_build(pd, po, np);
        if (!h) bad++;
        const uint64_t chunks[] = {1, 7, 64, 1u << 20};
        for (int c = 0; c < 4 && h; c++) {
            uint64_t *ka = NULL, ca = 0;
            if (orc_ac_scan(h, text, n, a, chunks[c], 1 + (c % 3), &ka, &ca)) bad++;
            if (ca != cb || (ca && memcmp(ka, kb, ca * 8))) bad++;
            orc_free(ka);
        }
        orc_ac_free(h);
        orc_free(kb);
        free(text);
        free(pd);
        free(po);
    }
    if (bad) {
        fprintf(stderr, "%d disagreements\n", bad);
        return 1;
    }
    printf("oracle sanitize: all checks passed\n");
    return 0;
}

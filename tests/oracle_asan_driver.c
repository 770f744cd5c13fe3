/* Drives the CPU oracle under AddressSanitizer / UBSan: exact-size heap
 * buffers (so any read or write past an end traps) for every tail length,
 * several AAD and IV lengths and every truncated tag length; prints one line
 * per case (the ciphertext's FNV-1a hash and the tag) for comparison with
 * the normally built oracle. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_gcm_encrypt(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len, const uint8_t *aad,
                       uint64_t aad_len, const uint8_t *pt, uint64_t len, uint8_t *ct, uint8_t tag[16]);
int oracle_gcm_decrypt_verify_t(const uint8_t *key, size_t key_len, const uint8_t *iv, size_t iv_len,
                                const uint8_t *aad, uint64_t aad_len, const uint8_t *ct, uint64_t len,
                                const uint8_t *tag, size_t tag_len, uint8_t *pt, int *accept);

static uint8_t *filled(size_t n, uint32_t seed)
{
    uint8_t *p = (uint8_t *)malloc(n ? n : 1);
    for (size_t i = 0; i < n; i++) {
        seed = seed * 1664525u + 1013904223u;
        p[i] = (uint8_t)(seed >> 24);
    }
    return p;
}

static uint64_t fnv(const uint8_t *p, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; i++)
        h = (h ^ p[i]) * 1099511628211ull;
    return h;
}

int main(void)
{
    static const size_t iv_lens[] = {12, 1, 8, 16, 60};
    static const size_t aad_lens[] = {0, 1, 16, 33};
    static const size_t tag_lens[] = {16, 15, 14, 13, 12, 8, 4};
    int cases = 0;
    for (size_t len = 0; len <= 70; len++) {
        const size_t key_len = 16 + 8 * (len % 3);
        const size_t iv_len = iv_lens[len % 5], aad_len = aad_lens[len % 4], tag_len = tag_lens[len % 7];
        uint8_t *key = filled(key_len, 1 + (uint32_t)len), *iv = filled(iv_len, 2 + (uint32_t)len);
        uint8_t *aad = filled(aad_len, 3 + (uint32_t)len), *pt = filled(len, 4 + (uint32_t)len);
        uint8_t *ct = (uint8_t *)malloc(len ? len : 1), *back = (uint8_t *)malloc(len ? len : 1);
        uint8_t tag[16];
        if (oracle_gcm_encrypt(key, key_len, iv, iv_len, aad_len ? aad : NULL, aad_len, len ? pt : NULL, len,
                               len ? ct : NULL, tag))
            return 2;
        uint8_t *t = (uint8_t *)malloc(tag_len);
        memcpy(t, tag, tag_len);
        int ok = -1;
        if (oracle_gcm_decrypt_verify_t(key, key_len, iv, iv_len, aad_len ? aad : NULL, aad_len, len ? ct : NULL,
                                        len, t, tag_len, len ? back : NULL, &ok) || ok != 1 ||
            (len && memcmp(back, pt, len)))
            return 3;
        t[tag_len - 1] ^= 1;
        if (oracle_gcm_decrypt_verify_t(key, key_len, iv, iv_len, aad_len ? aad : NULL, aad_len, len ? ct : NULL,
                                        len, t, tag_len, len ? back : NULL, &ok) || ok != 0)
            return 4;
        printf("%zu %zu %zu %zu %016llx ", len, key_len, iv_len, aad_len, (unsigned long long)fnv(ct, len));
        for (int k = 0; k < 16; k++)
            printf("%02x", tag[k]);
        printf("\n");
        free(key), free(iv), free(aad), free(pt), free(ct), free(back), free(t);
        cases++;
    }
    fprintf(stderr, "%d cases\n", cases);
    return 0;
}

// Packed attribute words.  An index packs its m attribute codes (Def. 1;
// ordinal codes, Sec. 3.2) into one 32-bit word, b bits per attribute,
// attribute i in bits b*i .. b*i + b - 1, with b the largest of 8, 4, 2, 1
// such that m * b <= 32 (see attr_bits).  Object codes must leave the
// all-ones field value free.  A query packs its constrained attributes the
// same way with a mask of their fields; a query code that no object can
// hold becomes the all-ones field, which never matches.  chi (Eq. 4-5)
// counts the masked fields that differ.
#pragma once

#include <cstdint>

namespace nhq {

// high bit of every b-bit field (b in {1, 2, 4, 8})
__host__ __device__ inline uint32_t attr_hmask(int b)
{
    return b == 8 ? 0x80808080u : b == 4 ? 0x88888888u : b == 2 ? 0xAAAAAAAAu : 0xFFFFFFFFu;
}

// fields 0 .. m-1
__host__ __device__ inline uint32_t attr_full_mask(int m, int b)
{
    return m * b >= 32 ? 0xFFFFFFFFu : ((1u << (m * b)) - 1u);
}

// number of differing fields of a and q under the field mask qm
__device__ __forceinline__ int chi_of(uint32_t a, uint32_t q, uint32_t qm, uint32_t hmask)
{
    const uint32_t x = (a ^ q) & qm;
    const uint32_t lo = ~hmask;
    const uint32_t y = ((x & lo) + lo) | x;
    return __popc(y & hmask);
}

// pack query codes (0xFF: wildcard); codes above the objects' range become
// the all-ones field
__host__ __device__ inline void attr_pack_query(const uint8_t *codes, int m, int b, uint32_t &word,
                                                uint32_t &mask)
{
    word = 0;
    mask = 0;
    const uint32_t fm = (b >= 32) ? 0xFFFFFFFFu : ((1u << b) - 1u);
    for (int i = 0; i < m; ++i) {
        const uint32_t c = codes[i];
        if (c == 0xFFu)
            continue;
        word |= (c < fm ? c : fm) << (b * i);
        mask |= fm << (b * i);
    }
}

// bits per attribute for m attributes whose object codes reach max_code:
// the largest b in {8, 4, 2, 1} with m * b <= 32, provided its fields keep
// the all-ones value free (max_code + 2 <= 2^b); 0 otherwise
inline int attr_bits(int m, int max_code)
{
    int b = 8;
    while (b > 1 && m * b > 32)
        b /= 2;
    if (m * b > 32 || max_code + 2 > (1 << b))
        return 0;
    return b;
}

}  // namespace nhq

// Edit distance (unit-cost insertions, deletions and substitutions) of a
// pattern of m <= 64*W characters against a text, by the bit-vector form of
// the dynamic programme (G. Myers, J. ACM 46(3), 1999; the variant for the
// distance of two whole strings as given by H. Hyyrö, 2001).  Column j of the
// table D (pattern prefixes down, text prefixes across) is held as two bit
// vectors of vertical differences, VP (D[i][j] - D[i-1][j] = +1) and VN
// (= -1); one text character updates all m cells with a few word
// operations.  For the distance of whole strings the top row is D[0][j] = j,
// so the horizontal difference entering row 1 is always +1: a 1 is shifted
// into HP.  The bottom cell D[m][j] is tracked in score from bit m-1 of the
// horizontal differences.  With W words the vectors are one 64W-bit integer:
// the addition carries and the shifts pass from word b to word b+1; nothing
// flows downward, so bits above m-1 never affect the result.
//
// peq[c * W + b] is word b of the match mask of byte value c (bit i set iff
// pattern character i equals c).
#pragma once

#include <cstdint>

namespace genie {

template <int W>
struct BitVectorEd {
    uint64_t vp[W], vn[W];
    uint32_t score;
    uint32_t top;        // word holding bit m-1
    uint64_t topbit;

    __host__ __device__ inline void init(uint32_t m) {
#pragma unroll
        for (int b = 0; b < W; b++) {
            vp[b] = ~0ull;
            vn[b] = 0;
        }
        score = m;
        top = (m - 1) >> 6;
        topbit = 1ull << ((m - 1) & 63);
    }

    // One text character: pm points at the W words of its match mask.
    __host__ __device__ inline void step(const uint64_t *pm) {
        uint64_t add_carry = 0;
        uint64_t hp_in = 1, hn_in = 0;
#pragma unroll
        for (int b = 0; b < W; b++) {
            if ((uint32_t)b > top)
                break;
            const uint64_t eq = pm[b];
            const uint64_t v_p = vp[b], v_n = vn[b];
            const uint64_t x = eq & v_p;
            uint64_t sum = x + v_p;
            const uint64_t c1 = sum < x ? 1ull : 0ull;
            sum += add_carry;
            const uint64_t c2 = sum < add_carry ? 1ull : 0ull;
            add_carry = c1 | c2;
            const uint64_t d0 = (sum ^ v_p) | eq | v_n;
            uint64_t hp = v_n | ~(d0 | v_p);
            uint64_t hn = v_p & d0;
            if ((uint32_t)b == top) {
                score += (hp & topbit) ? 1u : 0u;
                score -= (hn & topbit) ? 1u : 0u;
            }
            const uint64_t hp_out = hp >> 63, hn_out = hn >> 63;
            hp = (hp << 1) | hp_in;
            hn = (hn << 1) | hn_in;
            hp_in = hp_out;
            hn_in = hn_out;
            vp[b] = hn | ~(d0 | hp);
            vn[b] = hp & d0;
        }
    }
};

}  // namespace genie

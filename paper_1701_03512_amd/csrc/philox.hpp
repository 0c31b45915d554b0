// Philox4x32-10 counter-based generator for the device code of libbt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bt {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds; each round
// multiplies words 0 and 2 by the round multipliers, keeps the high halves
// xored with the other words and the key, and swaps; the key advances by
// the Weyl increments between rounds.
struct Ph4 {
    uint32_t v[4];
};

// BIAS: the output words come back xor 0x80008000 (each 16-bit half offset
// by 2^15, which maps unsigned halves onto signed ones in order); words 0
// and 2 take it through the last round's key words, at no cost.
template <bool BIAS = false>
__device__ __forceinline__ Ph4 philox10(uint32_t c0, uint32_t c1, uint32_t c2,
                                        uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (BIAS && r == 9) {
            k0 ^= 0x80008000u;
            k1 ^= 0x80008000u;
        }
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        // A three-input xor of two lane-varying words is one gfx950 bitop3
        // instruction (truth table 0x96 = a ^ b ^ c); where two of the
        // inputs are wave-uniform, plain xors let them combine on the scalar
        // unit first.  With the Monte Carlo counters (block and draw index
        // uniform over the wave, the stratum per lane) the state is partly
        // uniform through round 1, and in round 2 word 0's other inputs
        // still are; from round 3 on every word differs between lanes.
        uint32_t n0, n2;
        if (r < 2) {
            n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        } else if (r == 2) {
            n0 = (uint32_t)(m1 >> 32) ^ c1 ^ k0;
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c3, k1, 0x96);
        } else {
            n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(m1 >> 32), c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(m0 >> 32), c3, k1, 0x96);
        }
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    if (BIAS) {
        c1 ^= 0x80008000u;
        c3 ^= 0x80008000u;
    }
    return Ph4{{c0, c1, c2, c3}};
}

// Bernoulli steps from 16-bit half-words.  Suffix step j reads the half
// h_j of word (j % 8) / 2 of the block with counter (j / 8, m, z, stream)
// (high half for even j, low half for odd j) and goes up iff h_j is below
// the high half of thr = floor(p 2^32); on a tie it goes up iff g_j, the
// high half of word 0 of the block with counter (2^31 + j, m, z, stream),
// is below thr's low half.  The step's uniform is the 32-bit (h_j, g_j), so
// P(up) = thr / 2^32 exactly, and one block serves eight steps.
//
// step_keys8 fills k[i], i < n <= 8, for steps j = 8 b + i, such that step
// j goes up iff k[i] < 0: k = h_j - thr_hi, or g_j - thr_lo where h_j ties
// (about one step in 65536; then the wave draws the fallback blocks for
// its tied lanes).  The sign bit is the step's up bit.
__device__ __forceinline__ void step_keys8(uint32_t b, int n, uint32_t m, uint32_t z,
                                           uint32_t stream, uint32_t k0, uint32_t k1,
                                           uint32_t thr, int32_t (&k)[8])
{
    const Ph4 w = philox10(b, m, z, stream, k0, k1);
    const int32_t thi = (int32_t)(thr >> 16), tlo = (int32_t)(thr & 0xFFFFu);
    uint32_t kmin = 0xFFFFFFFFu;  // zero iff a used step ties (min3 chains)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t x = w.v[i >> 1];
        k[i] = (int32_t)((i & 1) ? (x & 0xFFFFu) : (x >> 16)) - thi;
        if (i < n) kmin = min(kmin, (uint32_t)k[i]);
    }
    if (kmin == 0u) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if (i < n && k[i] == 0)
                k[i] = (int32_t)(philox10(0x80000000u + 8u * b + (uint32_t)i, m, z, stream, k0, k1).v[0] >> 16) - tlo;
    }
}


typedef short short2_t __attribute__((ext_vector_type(2)));
typedef unsigned short ushort2_t __attribute__((ext_vector_type(2)));

// The up bits of the eight steps j = 8 b + i of one Philox block (bit i set
// iff step j goes up): the decisions of step_keys8, two steps per
// instruction.  With every half-word h and thr's high half offset by 2^15
// (signed view, same order), one saturating packed subtraction per word
// gives two differences whose sign bits are the two steps' up bits
// (saturation keeps the sign, and only a tie gives zero); one byte permute
// per pair of words spreads four sign bits over four bytes (0x00 / 0xFF),
// and two signed byte dot products weigh them into the 8-bit pattern.  A tie (h_j equal to thr's high half) is settled by the fallback
// block of step_keys8.
__device__ __forceinline__ uint32_t up_bits8(uint32_t b, uint32_t m, uint32_t z, uint32_t stream,
                                             uint32_t k0, uint32_t k1, uint32_t thr)
{
    const Ph4 w = philox10<true>(b, m, z, stream, k0, k1);
    const uint32_t t16 = (thr >> 16) ^ 0x8000u;
    const short2_t t = __builtin_bit_cast(short2_t, t16 | (t16 << 16));
    uint32_t d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        d[q] = __builtin_bit_cast(uint32_t,
                                  __builtin_elementwise_sub_sat(__builtin_bit_cast(short2_t, w.v[q]), t));
    // bytes, in step order: sign of bit 31 (high half, even step) and of
    // bit 15 (low half, odd step) of the first word, then of the second;
    // each byte is 0 or -1 (0xFF) as a signed 8-bit number
    const uint32_t s01 = __builtin_amdgcn_perm(d[1], d[0], 0x0A0B0809u);
    const uint32_t s23 = __builtin_amdgcn_perm(d[3], d[2], 0x0A0B0809u);
    // a signed four-byte dot product with the weights -2^i turns them into
    // the pattern: bytes (-1, -2, -4, -8) for steps 0-3, (-16, -32, -64,
    // -128) for steps 4-7
    uint32_t bits = (uint32_t)__builtin_amdgcn_sdot4((int)s23, (int)0x80C0E0F0u, 0, false);
    bits = (uint32_t)__builtin_amdgcn_sdot4((int)s01, (int)0xF8FCFEFFu, (int)bits, false);
    // a zero half is a tie: unsigned minimum over the halves
    const ushort2_t mn = __builtin_elementwise_min(
        __builtin_elementwise_min(__builtin_bit_cast(ushort2_t, d[0]), __builtin_bit_cast(ushort2_t, d[1])),
        __builtin_elementwise_min(__builtin_bit_cast(ushort2_t, d[2]), __builtin_bit_cast(ushort2_t, d[3])));
    if (mn.x == 0 || mn.y == 0) {
        const uint32_t tlo = thr & 0xFFFFu;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t half = (i & 1) ? (d[i >> 1] & 0xFFFFu) : (d[i >> 1] >> 16);
            if (half == 0u) {
                const uint32_t g =
                    philox10(0x80000000u + 8u * b + (uint32_t)i, m, z, stream, k0, k1).v[0] >> 16;
                bits = (bits & ~(1u << i)) | ((g < tlo ? 1u : 0u) << i);
            }
        }
    }
    return bits;
}

}  // namespace bt

// ldp_device.hpp -- device building blocks of the gfx950 LDP kernels.
//
// One lane is a "column worker": it owns 8 adjacent code columns of one image
// and walks down a range of code rows with a three-row register window, so
// every image byte it needs is loaded once per row (plus a one-byte halo on
// each side, loaded in the same dwords).
//
// Arithmetic (exact integers throughout):
//   * Section 2.3 removes the redundancy of the eight 3x3 mask products by
//     sharing column partial sums between masks (Eqs. 7-29).  Taken to its
//     end, every Kirsch response is m_i = 8*S_i - 3*T, where S_i is the sum of
//     the three ring neighbours that mask i weighs with +5 (ring order E, NE,
//     N, NW, W, SW, S, SE; S_i = p_{i-1} + p_i + p_{i+1}) and T is the sum of
//     all eight neighbours.  T is common to the eight responses of a pixel, so
//     the order of the responses, the k-th largest one and every tie are
//     those of the S_i.  The code of Eqs. 2-3 is therefore computed from the
//     S_i alone: bit i is set when S_i >= (k-th largest S).
//   * The S_i of neighbouring pixels share partial sums: S0 and S4 are column
//     3-sums (the right and left columns), S2 and S6 are row 3-sums (the rows
//     above and below), and the four corner triples are three pixels each.
//     Each column 3-sum serves two pixels, each row 3-sum two code rows.
//     Every sum is one three-input add (v_add3_u32): one issue slot where
//     chains of two-input adds over shared pair sums take more.
//   * S_i <= 765 fits 16 bits, so two pixels share one 32-bit register.  No
//     sum can carry out of its 16-bit field, so sums are plain 32-bit adds;
//     only min/max use packed 16-bit instructions.
//     The 8 pixels of a lane are held as four pairs (c, c+4), c = 0..3,
//     which makes the left and right neighbours of each pair another pair.
//   * The k-th largest of eight values is a branch-free min/max network
//     (for k = 3, a median of three values taken from four sorted pairs).
//   * The code bits are the sign bits of S_i + 0x8000 - t (bit 15 of a field
//     is set exactly when S_i >= t, and no field can carry): v_perm_b32
//     gathers four of them into four byte masks at once and v_bitop3_b32
//     merges the eight directions.  The codes stay in the two words the
//     gather makes (pixels 0, 1, 4, 5 and 2, 3, 6, 7).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldp {

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// What a pixel's code is made from (a template argument of every kernel):
// the S_i, whose order is that of the signed responses m_i = 8*S_i - 3*T
// (Eq. 2 as written); |m_i| (ranking by response magnitude); the signed
// responses computed mask by mask (the unaccelerated route, same codes); or
// the LBP comparison with the centre pixel (pair_values below).
enum : int { RANK_SIGNED = 0, RANK_MAGNITUDE = 1, DIRECT_MASKS = 2, CODE_LBP = 3 };

__device__ __forceinline__ u16x2 V(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t U(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ u16x2 vmax(u16x2 a, u16x2 b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ u16x2 vmin(u16x2 a, u16x2 b) { return __builtin_elementwise_min(a, b); }

// Maximum and minimum of three, one instruction each (v_pk_maximum3_f16,
// v_pk_minimum3_f16).  The fields are compared as f16: a 16-bit pattern below
// 0x7C00 with the sign bit clear is a finite non-negative f16 (zero, denormal
// or normal), and such values are ordered exactly as their patterns, so the
// f16 maximum / minimum of sums <= 765 is their integer maximum / minimum.
// The kernels keep f16 denormals (the default mode), and IEEE maximum and
// minimum return one of their operands unchanged.
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h16x2 H(u16x2 v) { return __builtin_bit_cast(h16x2, v); }
__device__ __forceinline__ u16x2 vmax3(u16x2 a, u16x2 b, u16x2 c)
{
    return __builtin_bit_cast(
        u16x2, __builtin_elementwise_maximum(__builtin_elementwise_maximum(H(a), H(b)), H(c)));
}
__device__ __forceinline__ u16x2 vmin3(u16x2 a, u16x2 b, u16x2 c)
{
    return __builtin_bit_cast(
        u16x2, __builtin_elementwise_minimum(__builtin_elementwise_minimum(H(a), H(b)), H(c)));
}

// ------------------------------------------------------------ k-th largest
// Eq. 2's m_k: the k-th element of the eight values in descending order,
// duplicates kept.  The values are first sorted in four pairs: h_j / l_j are
// the larger / smaller of pair j (h0, h1, g0, g1 and l0, l1, k0, k1).  A pair
// puts 0, 1 or 2 values at or above any level x, and x is at most the k-th
// largest exactly when a + o >= k, with o the number of pairs whose larger
// value reaches x and a the number whose smaller one does (a pair counted in
// a is counted in o).  Written with min/max (each level test is monotone, so
// a network right for every level is right for every input):
//   k = 2: o >= 2 or a >= 1: the largest of the pair minima and the second
//          largest of the pair maxima;
//   k = 3: (o >= 2 and a >= 1) or o >= 3: the median of three values, the
//          second and third largest of the pair maxima and the largest pair
//          minimum;
//   k = 4: a >= 2, or a >= 1 and o >= 3, or o = 4.
// The four pair maxima are ranked as two sorted pairs (x1 >= v from h0, h1;
// y1 >= z from g0, g1): the largest is max(x1, y1), the second and third are
// max(min(x1, y1), v, z) and min(x1, y1, max(v, z)), the smallest min(v, z).
// The (9-k)-th largest is the k-th smallest: the same networks with max and
// min exchanged (k = 5, 6, 7 from 4, 3, 2).
template <bool SMALLEST>
struct Order {
    static __device__ __forceinline__ u16x2 hi(u16x2 a, u16x2 b) { return SMALLEST ? vmin(a, b) : vmax(a, b); }
    static __device__ __forceinline__ u16x2 lo(u16x2 a, u16x2 b) { return SMALLEST ? vmax(a, b) : vmin(a, b); }
    static __device__ __forceinline__ u16x2 hi3(u16x2 a, u16x2 b, u16x2 c)
    {
        return SMALLEST ? vmin3(a, b, c) : vmax3(a, b, c);
    }
    static __device__ __forceinline__ u16x2 lo3(u16x2 a, u16x2 b, u16x2 c)
    {
        return SMALLEST ? vmax3(a, b, c) : vmin3(a, b, c);
    }
};

// k-th largest (SMALLEST = false) or k-th smallest (true) for k = 2, 3, 4:
// 16, 19 and 24 packed min/max per pixel pair
template <int K, bool SMALLEST>
__device__ __forceinline__ u16x2 kth_network(const u16x2 (&s)[8])
{
    typedef Order<SMALLEST> O;
    const u16x2 h0 = O::hi(s[0], s[1]), l0 = O::lo(s[0], s[1]);
    const u16x2 h1 = O::hi(s[2], s[3]), l1 = O::lo(s[2], s[3]);
    const u16x2 g0 = O::hi(s[4], s[5]), k0 = O::lo(s[4], s[5]);
    const u16x2 g1 = O::hi(s[6], s[7]), k1 = O::lo(s[6], s[7]);
    const u16x2 x1 = O::hi(h0, h1), v = O::lo(h0, h1);
    const u16x2 y1 = O::hi(g0, g1), z = O::lo(g0, g1);
    if constexpr (K == 2) {
        // max(l0, l1, k0, k1, min(x1, y1), v, z)
        return O::hi3(O::hi3(l0, l1, k0), O::hi3(k1, v, z), O::lo(x1, y1));
    } else if constexpr (K == 3) {
        // median(p, q, r) with p = min(x1, y1), r = max(v, z) (the middle two
        // of the pair maxima, either order) and q the largest pair minimum,
        // as max(min(p, max(q, r)), min(q, r)); max(q, r) = max(q, v, z)
        const u16x2 q = O::hi3(l0, l1, O::hi(k0, k1));
        const u16x2 r = O::hi(v, z);
        return O::hi(O::lo3(x1, y1, O::hi3(q, v, z)), O::lo(q, r));
    } else {
        static_assert(K == 4, "k = 2, 3, 4");
        // max(min(a1, o3), a2, o4): a1 >= a2 the two largest pair minima, o3
        // and o4 the third and fourth largest pair maxima
        const u16x2 ma = O::hi(l0, l1), na = O::lo(l0, l1);
        const u16x2 mb = O::hi(k0, k1), nb = O::lo(k0, k1);
        const u16x2 a1 = O::hi(ma, mb);
        const u16x2 o3 = O::lo3(x1, y1, O::hi(v, z)), o4 = O::lo(v, z);
        // a2 = max(na, nb, min(ma, mb))
        return O::hi3(O::hi3(O::lo(a1, o3), na, nb), O::lo(ma, mb), o4);
    }
}

template <int K>
__device__ __forceinline__ u16x2 kth_largest(const u16x2 (&s)[8])
{
    static_assert(K >= 1 && K <= 8, "k in 1..8");
    if constexpr (K == 1)
        return vmax3(vmax3(s[0], s[1], s[2]), vmax3(s[3], s[4], s[5]), vmax(s[6], s[7]));
    else if constexpr (K == 8)
        return vmin3(vmin3(s[0], s[1], s[2]), vmin3(s[3], s[4], s[5]), vmin(s[6], s[7]));
    else if constexpr (K <= 4)
        return kth_network<K, false>(s);
    else
        return kth_network<9 - K, true>(s);
}

// Sum of three words holding two 16-bit fields each (no field carries): one
// v_add3_u32, written as an instruction so that the compiler does not turn
// the sums back into chains of two-input adds over shared partial sums.
__device__ __forceinline__ uint32_t add3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_add3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// ------------------------------------------------------------ image rows
// One image row as seen by a lane: bytes B[0..9] = image columns j0..j0+9,
// held as six pairs X[a] = (B[a], B[a+4]).  Pixel pair c (c = 0..3) is
// centred on X[c+1]; its left and right neighbour columns are X[c] and
// X[c+2].  R[c] is the row 3-sum of pair c.
struct Row {
    uint32_t X[6];
    uint32_t R[4];
};

__device__ __forceinline__ uint32_t pair_sel(int a)
{
    // bytes: [lo.a, 0, hi.a, 0] from {src0 = hi word, src1 = lo word}
    return (uint32_t)a | (0x0Cu << 8) | ((uint32_t)(4 + a) << 16) | (0x0Cu << 24);
}

// With RANK_MAGNITUDE the pairs hold 8 * byte, so every sum below is 8 times
// the pixel sum (8 * S_i <= 6120, 8 * T <= 16320: still no carry).
template <int MODE>
__device__ __forceinline__ void make_row(Row &r, uint32_t u0, uint32_t u1, uint32_t u2)
{
    r.X[0] = __builtin_amdgcn_perm(u1, u0, pair_sel(0));
    r.X[1] = __builtin_amdgcn_perm(u1, u0, pair_sel(1));
    r.X[2] = __builtin_amdgcn_perm(u1, u0, pair_sel(2));
    r.X[3] = __builtin_amdgcn_perm(u1, u0, pair_sel(3));
    r.X[4] = __builtin_amdgcn_perm(u2, u1, pair_sel(0));
    r.X[5] = __builtin_amdgcn_perm(u2, u1, pair_sel(1));
    if constexpr (MODE == RANK_MAGNITUDE) {
#pragma unroll
        for (int a = 0; a < 6; ++a)
            r.X[a] <<= 3;  // fields <= 255 * 8: nothing crosses into the next field
    }
    // two 16-bit fields per add; no field exceeds 765, so nothing carries
#pragma unroll
    for (int c = 0; c < 4; ++c)
        r.R[c] = add3(r.X[c], r.X[c + 1], r.X[c + 2]);
}

// Raw words of one row: 16 bytes starting at the 4-aligned offset at or
// below the lane's first byte, plus the shift s (0..3) to that byte.
struct RawRow {
    uint32_t w[4];
    uint32_t s;
};

// ------------------------------------------------------------ mask taps
// One tap of a direct mask correlation on two 16-bit fields: acc + w * x per
// field (modulo 2^16, exact here), w = +5 or -3 as an inline constant for both
// fields.  Written as instructions so that the compiler cannot merge the taps
// of different masks into shared sums: the direct route must do all 8 per
// response.
__device__ __forceinline__ uint32_t mad_w5(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_pk_mad_u16 %0, %1, 5, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}
__device__ __forceinline__ uint32_t mad_wm3(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_pk_mad_u16 %0, %1, -3, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// ------------------------------------------------------------ one code row
// The eight values a pixel pair compares and the threshold they are compared
// with, per mode:
//   RANK_SIGNED     S_i (the order of m_i = 8*S_i - 3*T), threshold the k-th
//                   largest S (Eqs. 2-3);
//   RANK_MAGNITUDE  |m_i| = |8*S_i - 3*T|, threshold the k-th largest;
//   DIRECT_MASKS    m_i + 3825 computed mask by mask as Eq. 1's 8-tap
//                   correlation (weights +5 and -3, one multiply-add per tap,
//                   no shared sums: the unaccelerated computation), threshold
//                   the k-th largest -- the same codes as RANK_SIGNED;
//   CODE_LBP        the eight neighbours, threshold the centre (Section 2.1).
// Every value is below 0x8000 - threshold + 0x8000, so bit 15 of each field
// of value + (0x8000 - threshold) is set exactly when value >= threshold.
template <int K, int MODE>
__device__ __forceinline__ void pair_values(const Row &t, const Row &m, const Row &b,
                                            const uint32_t (&col)[6], int c, uint32_t (&S)[8],
                                            uint32_t &bias)
{
    const int a = c + 1;  // the pair's centre column pair
    if constexpr (MODE == CODE_LBP) {
        S[0] = m.X[a + 1];  // E
        S[1] = t.X[a + 1];  // NE
        S[2] = t.X[a];      // N
        S[3] = t.X[a - 1];  // NW
        S[4] = m.X[a - 1];  // W
        S[5] = b.X[a - 1];  // SW
        S[6] = b.X[a];      // S
        S[7] = b.X[a + 1];  // SE
        bias = 0x80008000u - m.X[a];
        return;
    } else {
        if constexpr (MODE == DIRECT_MASKS) {
            // neighbours in ring order E, NE, N, NW, W, SW, S, SE; mask i
            // weighs neighbours i-1, i, i+1 with +5 and the rest with -3
            const uint32_t P[8] = {m.X[a + 1], t.X[a + 1], t.X[a],     t.X[a - 1],
                                   m.X[a - 1], b.X[a - 1], b.X[a],     b.X[a + 1]};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                uint32_t acc = 0x0EF10EF1u;  // 3825 per field: m_i + 3825 stays in 0..7650
                // taps from neighbour i round the ring: no two masks share a
                // chain prefix, so no tap is computed once for several masks
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int j = (i + d) % 8;
                    acc = (d == 0 || d == 1 || d == 7) ? mad_w5(P[j], acc) : mad_wm3(P[j], acc);
                }
                S[i] = acc;
            }
        } else {
            S[0] = col[a + 1];                          // E   column to the right
            S[1] = add3(m.X[a + 1], t.X[a + 1], t.X[a]);  // NE  E + NE + N
            S[2] = t.R[c];                              // N   row above
            S[3] = add3(t.X[a], t.X[a - 1], m.X[a - 1]);  // NW  N + NW + W
            S[4] = col[a - 1];                          // W   column to the left
            S[5] = add3(m.X[a - 1], b.X[a - 1], b.X[a]);  // SW  W + SW + S
            S[6] = b.R[c];                              // S   row below
            S[7] = add3(b.X[a], b.X[a + 1], m.X[a + 1]);  // SE  S + SE + E
            if constexpr (MODE == RANK_MAGNITUDE) {
                // the sums are 8 * S_i and 8 * T (scaled rows); 3 * T is
                // ((8 * T) >> 3) * 3 (the low 3 bits of each field are 0, so
                // the shift moves nothing across fields), and
                // |m_i| = |8 * S_i - 3 * T| = max - min per field
                const uint32_t T8 = add3(col[a + 1], col[a - 1], t.X[a] + b.X[a]);
                const uint32_t T1 = T8 >> 3;
                const u16x2 T3 = V((T1 << 1) + T1);
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    S[i] = U(vmax(V(S[i]), T3)) - U(vmin(V(S[i]), T3));
            }
        }
        u16x2 Sv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            Sv[i] = V(S[i]);
        bias = 0x80008000u - U(kth_largest<K>(Sv));  // 0x8000 - threshold per field
    }
}

// Codes of the lane's 8 pixels for the code row whose image rows are t
// (above), m (centre) and b (below): byte p of q0 is the code of pixel
// (0, 1, 4, 5)[p], byte p of q1 that of pixel (2, 3, 6, 7)[p].
template <int K, int MODE>
__device__ __forceinline__ void code_row(const Row &t, const Row &m, const Row &b, uint32_t &q0,
                                         uint32_t &q1)
{
    if constexpr (K == 8 && MODE != CODE_LBP) {
        // the 8th largest is the minimum: every response reaches it
        q0 = q1 = 0xFFFFFFFFu;
        return;
    } else {
        uint32_t col[6];
#pragma unroll
        for (int a = 0; a < 6; ++a)
            col[a] = add3(t.X[a], m.X[a], b.X[a]);

        // Two halves: pixel pairs (0, 1) give the codes of pixels 0, 1, 4, 5;
        // pairs (2, 3) those of pixels 2, 3, 6, 7.
        uint32_t code[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t S[2][8], bias[2];
#pragma unroll
            for (int e = 0; e < 2; ++e)
                pair_values<K, MODE>(t, m, b, col, 2 * h + e, S[e], bias[e]);
            // bit 15 of a field of S_i + bias is set iff S_i >= threshold.
            // The 16 adds are kept together (scheduling barriers around
            // them): on gfx950 a run of independent 32-bit adds issues faster
            // than adds spread between other instructions.
            uint32_t x[2][8];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    x[e][i] = S[e][i] + bias[e];
            __builtin_amdgcn_sched_barrier(0);
            // v_perm_b32 turns the four sign bits of a direction into byte
            // masks [first pair lo, second pair lo, first hi, second hi], and
            // bit i of every byte is taken from direction i.
            uint32_t acc = __builtin_amdgcn_perm(x[1][0], x[0][0], 0x0B090A08u);
#pragma unroll
            for (int i = 1; i < 8; ++i) {
                const uint32_t msk = __builtin_amdgcn_perm(x[1][i], x[0][i], 0x0B090A08u);
                acc = __builtin_amdgcn_bitop3_b32(0x01010101u << i, msk, acc, 0xCA);
            }
            code[h] = acc;
        }
        q0 = code[0];
        q1 = code[1];
    }
}

// Code of pixel p (0..7) from the two code words of code_row.
__device__ __forceinline__ uint32_t code_of(uint32_t q0, uint32_t q1, int p)
{
    return (((p & 2) ? q1 : q0) >> (8 * ((p & 1) | ((p >> 1) & 2)))) & 0xFFu;
}

}  // namespace ldp

// Device-side lookup UTF-8 validation (Keiser & Lemire, section 6), four bytes
// per 32-bit register ("SWAR"), for gfx950.
//
// Byte k of a register holds stream position 4*j + k (little-endian).  For a
// register x and the register p that precedes it in the stream:
//
//   prev1 = the stream shifted by one byte   (section 6.1; v_alignbyte_b32)
//   byte_1_high[prev1 >> 4] & byte_1_low[prev1 & 15] & byte_2_high[x >> 4]
//                                            (section 6.1, three 16-entry tables)
//   ^ must23                                 (section 6.2: 0x80 where the byte two
//                                             back is >= 0xE0 or three back >= 0xF0)
//
// A non-zero byte of the result marks a position where the input is not UTF-8.
//
// The tables are the paper's three nibble tables (bit order of Table 9; their
// contents follow from the error patterns of Table 8):
//
//   byte_1_high  02 02 02 02 02 02 02 02 80 80 80 80 21 01 15 49
//   byte_1_low   E7 A3 83 83 8B CB CB CB CB CB CB CB CB DB CB CB
//   byte_2_high  01 01 01 01 01 01 01 01 E6 AE BA BA 01 01 01 01
//
// A 16-entry lookup of four bytes at once is done with v_perm_b32, which picks
// bytes out of an 8-byte pool: the low three bits of a nibble select within a
// half-table and bit 3 picks the half.  byte_1_high and byte_2_high have a
// constant low half (0x02 and 0x01), so one v_perm_b32 on the high half is
// merged with the constant under a sign-bit mask; byte_1_low needs both halves,
// merged by a second v_perm_b32.  v_perm_b32's selectors 8..11 return the sign
// of pool bytes 1, 3, 5, 7 spread over a whole byte, which turns a pair of
// shifted registers into a 0x00/0xFF sign mask in one instruction.  v_lerp_u8
// computes (a + b) >> 1 per byte without carries between bytes, so bit 7 of
// lerp(v, 0x20) is exactly "v >= 0xE0" (the unsigned comparisons of sections
// 6.2-6.3).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace utf8v {

// Pools: v_perm_b32(hi, lo, sel) picks byte sel (0..7) of the 64-bit value hi:lo.
constexpr uint32_t kB1H_HI_LO = 0x80808080u;  // byte_1_high[8..11]
constexpr uint32_t kB1H_HI_HI = 0x49150121u;  // byte_1_high[12..15]
constexpr uint32_t kB1L_LO_LO = 0x8383A3E7u;  // byte_1_low[0..3]
constexpr uint32_t kB1L_LO_HI = 0xCBCBCB8Bu;  // byte_1_low[4..7]
constexpr uint32_t kB1L_HI_LO = 0xCBCBCBCBu;  // byte_1_low[8..11]
constexpr uint32_t kB1L_HI_HI = 0xCBCBDBCBu;  // byte_1_low[12..15]
constexpr uint32_t kB2H_HI_LO = 0xBABAAEE6u;  // byte_2_high[8..11]
constexpr uint32_t kB2H_HI_HI = 0x01010101u;  // byte_2_high[12..15]
constexpr uint32_t kB1H_LOW_HALF = 0x02020202u;  // byte_1_high[0..7]
constexpr uint32_t kB2H_LOW_HALF = 0x01010101u;  // byte_2_high[0..7]

// Selector turning (x, x shifted up one byte) into a per-byte sign mask.
constexpr uint32_t kSignSel = 0x0B090A08u;

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t align(uint32_t hi, uint32_t lo, uint32_t bytes) {
  return __builtin_amdgcn_alignbyte(hi, lo, bytes);
}
// Per byte: bit 7 of the result is set iff v >= 256 - k (k a byte constant).
__device__ __forceinline__ uint32_t ge_mask7(uint32_t v, uint32_t k) {
  return __builtin_amdgcn_lerp(v, k, 0u);
}
// v_bitop3_b32 computes any bitwise function of three operands; its 8-bit truth
// table is the function applied to a = 0xF0, b = 0xCC, c = 0xAA.  Each helper
// derives its table from its own formula at compile time.
#define UTF8V_BITOP3(A, B, C, EXPR)                                                              \
  __builtin_amdgcn_bitop3_b32((A), (B), (C),                                                    \
                              ([](uint32_t a, uint32_t b, uint32_t c) constexpr { return (EXPR) & 0xFFu; })( \
                                  0xF0u, 0xCCu, 0xAAu))

__device__ __forceinline__ uint32_t select_bits(uint32_t m, uint32_t x, uint32_t y) {  // m ? x : y, bitwise
  return UTF8V_BITOP3(m, x, y, (a & b) | (~a & c));
}
__device__ __forceinline__ uint32_t and3(uint32_t x, uint32_t y, uint32_t z) {
  return UTF8V_BITOP3(x, y, z, a & b & c);
}
__device__ __forceinline__ uint32_t or_and(uint32_t x, uint32_t y, uint32_t z) {  // (x | y) & z
  return UTF8V_BITOP3(x, y, z, (a | b) & c);
}
__device__ __forceinline__ uint32_t and_or(uint32_t x, uint32_t y, uint32_t z) {  // (x & y) | z
  return UTF8V_BITOP3(x, y, z, (a & b) | c);
}
__device__ __forceinline__ uint32_t or_xor(uint32_t acc, uint32_t x, uint32_t y) {  // acc | (x ^ y)
  return UTF8V_BITOP3(acc, x, y, a | (b ^ c));
}
__device__ __forceinline__ uint32_t or_andn(uint32_t x, uint32_t y, uint32_t z) {  // x | (y & ~z)
  return UTF8V_BITOP3(x, y, z, a | (b & ~c));
}
__device__ __forceinline__ uint32_t andn_and(uint32_t x, uint32_t y, uint32_t z) {  // x & ~y & z
  return UTF8V_BITOP3(x, y, z, a & ~b & c);
}

// The three table lookups of section 6.1 from prepared indices:
//   sh1 / sl1 / sh2: low 3 bits of prev1's high nibble, prev1's low nibble, the byte's high nibble;
//   neg1 / neg2:     0xFF where prev1 / the byte is >= 0x80 (bit 3 of the high nibble);
//   half:            byte k = k + 4 * (bit 3 of prev1's low nibble).
__device__ __forceinline__ uint32_t lookup3(uint32_t sh1, uint32_t sl1, uint32_t sh2, uint32_t neg1, uint32_t neg2,
                                            uint32_t half) {
  const uint32_t byte_1_high = select_bits(neg1, perm(kB1H_HI_HI, kB1H_HI_LO, sh1), kB1H_LOW_HALF);
  const uint32_t byte_1_low = perm(perm(kB1L_HI_HI, kB1L_HI_LO, sl1), perm(kB1L_LO_HI, kB1L_LO_LO, sl1), half);
  const uint32_t byte_2_high = select_bits(neg2, perm(kB2H_HI_HI, kB2H_HI_LO, sh2), kB2H_LOW_HALF);
  return and3(byte_1_high, byte_1_low, byte_2_high);
}

__device__ __forceinline__ uint32_t low_half_selector(uint32_t prev1) {
  return and_or(prev1 >> 1, 0x04040404u, 0x03020100u);
}

// Section 6.1: the classification byte of each position (AND of the three lookups).
// prev1 holds the byte before each position, prev2 the byte two before.
__device__ __forceinline__ uint32_t classify(uint32_t x, uint32_t prev1, uint32_t prev2) {
  return lookup3((prev1 >> 4) & 0x07070707u, prev1 & 0x07070707u, (x >> 4) & 0x07070707u,
                 perm(prev1, prev2, kSignSel), perm(x, prev1, kSignSel), low_half_selector(prev1));
}

// Section 6.2: 0x80 where a second continuation byte is required.
__device__ __forceinline__ uint32_t must23(uint32_t prev2, uint32_t prev3) {
  return or_and(ge_mask7(prev2, 0x20202020u), ge_mask7(prev3, 0x10101010u), 0x80808080u);
}

// Per-position error bytes of register x preceded by register p (sections 6.1-6.2).
__device__ __forceinline__ uint32_t position_errors(uint32_t x, uint32_t p) {
  const uint32_t prev1 = align(x, p, 3);
  const uint32_t prev2 = align(x, p, 2);
  const uint32_t prev3 = align(x, p, 1);
  return classify(x, prev1, prev2) ^ must23(prev2, prev3);
}

// Section 6.3 on the three bytes before a position: non-zero iff a character is
// still open there (last byte >= 0xC0, second-to-last >= 0xE0, third-to-last >= 0xF0).
// p holds those bytes in its top three bytes.
__device__ __forceinline__ uint32_t open_at_end(uint32_t p) {
  const uint32_t c = ge_mask7(p, 0x40404040u) & 0x80000000u;  // byte 3 >= 0xC0
  const uint32_t e = ge_mask7(p, 0x20202020u) & 0x00800000u;  // byte 2 >= 0xE0
  const uint32_t f = ge_mask7(p, 0x10101010u) & 0x00008000u;  // byte 1 >= 0xF0
  return c | e | f;
}

// ---- a run of consecutive registers ----------------------------------------------------
// Along a run, the sign masks, high-nibble indices and must23 inputs of a register
// are computed once and shifted in for the next register instead of being
// recomputed from the shifted bytes.

struct Carry {
  uint32_t neg2;  // sign mask of the bytes
  uint32_t sh2;   // low 3 bits of the high nibbles
  uint32_t g;     // bit 7 at byte j: b[j] >= 0xE0 or b[j-1] >= 0xF0
};

// Errors of the first register x of a run, preceded by p, ORed into acc; fills c for x.
__device__ __forceinline__ uint32_t errors_first(uint32_t acc, uint32_t x, uint32_t p, Carry& c) {
  const uint32_t prev1 = align(x, p, 3);
  const uint32_t prev2 = align(x, p, 2);
  const uint32_t prev3 = align(x, p, 1);
  c.neg2 = perm(x, prev1, kSignSel);
  c.sh2 = (x >> 4) & 0x07070707u;
  c.g = or_and(ge_mask7(x, 0x20202020u), ge_mask7(prev1, 0x10101010u), 0x80808080u);
  const uint32_t sc = lookup3((prev1 >> 4) & 0x07070707u, prev1 & 0x07070707u, c.sh2, perm(prev1, prev2, kSignSel),
                              c.neg2, low_half_selector(prev1));
  return or_xor(acc, sc, must23(prev2, prev3));
}

// Errors of register x following register xp in the run, ORed into acc (c holds xp's
// values; updated to x's).  must23 at position i equals g at position i-2.
__device__ __forceinline__ uint32_t errors_next(uint32_t acc, uint32_t x, uint32_t xp, Carry& c) {
  const uint32_t prev1 = align(x, xp, 3);
  const uint32_t neg2 = perm(x, prev1, kSignSel);
  const uint32_t sh2 = (x >> 4) & 0x07070707u;
  const uint32_t g = or_and(ge_mask7(x, 0x20202020u), ge_mask7(prev1, 0x10101010u), 0x80808080u);
  const uint32_t sc = lookup3(align(sh2, c.sh2, 3), prev1 & 0x07070707u, sh2, align(neg2, c.neg2, 3), neg2,
                              low_half_selector(prev1));
  acc = or_xor(acc, sc, align(g, c.g, 2));
  c.neg2 = neg2;
  c.sh2 = sh2;
  c.g = g;
  return acc;
}

// Errors of a 16-byte chunk (x0..x3) preceded by the dword p, ORed into acc.
__device__ __forceinline__ uint32_t chunk_errors(uint32_t acc, uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                 uint32_t p) {
  Carry c;
  acc = errors_first(acc, x0, p, c);
  acc = errors_next(acc, x1, x0, c);
  acc = errors_next(acc, x2, x1, c);
  return errors_next(acc, x3, x2, c);
}


// ---- text of 1- and 2-byte characters -----------------------------------------------------
// Where no byte of a position's window (the byte and the three before it) is >= 0xE0, the
// checks of 6.1-6.2 can only report a continuation byte that does not follow a lead
// (C0..DF), a lead that is not followed by a continuation, or a continuation after the
// overlong leads C0 and C1; must23 is zero.  The same positions are then non-zero in
//   (lead(prev1) ^ cont(byte)) | (prev1 is C0 or C1)
// (bit 7 of each byte; the other bits are left over from the comparisons).

// Bit 7 of each byte: the byte is >= 0xE0.
__device__ __forceinline__ uint32_t ge_e0(uint32_t v) { return ge_mask7(v, 0x20202020u); }

// Errors of register x preceded by register p (no byte >= 0xE0 in either): bit 7 of each
// byte marks an error at that position.
__device__ __forceinline__ uint32_t two_byte_errors(uint32_t x, uint32_t p) {
  const uint32_t prev1 = align(x, p, 3);
  const uint32_t lead = ge_mask7(prev1, 0x40404040u);                                 // prev1 >= 0xC0
  const uint32_t t = UTF8V_BITOP3(x, ge_mask7(x, 0x40404040u), lead, (a & ~b) ^ c);  // cont(x) ^ lead
  return UTF8V_BITOP3(t, lead, ge_mask7(prev1, 0x3E3E3E3Eu), a | (b & ~c));          // | prev1 in C0..C1
}

// ---- section 6.4's ASCII test, per tile ---------------------------------------------------
// A tile whose bytes (and the three before it) are all ASCII cannot hold an error.  The test
// is taken with an exponential back-off: after a tile that is not all ASCII it is skipped for
// 3, 7, 15, ... up to 63 tiles, and a tile that is all ASCII brings it back to every tile.
// Text without ASCII tiles pays for a handful of tests per wave, ASCII text skips every
// tile, and mixed text is tested about as often as it has ASCII tiles.
struct AsciiBackoff {
  int skip = 0;  // tiles to go before the next test (wave-uniform)
  int next = 3;  // skip after the next failed test
  __device__ __forceinline__ bool due() {
    if (skip == 0) return true;
    --skip;
    return false;
  }
  __device__ __forceinline__ void result(bool all_ascii) {
    if (all_ascii) {
      next = 3;
    } else {
      skip = next;
      next = next < 63 ? 2 * next + 1 : 63;
    }
  }
};

// ---- four streams across the byte lanes ------------------------------------------------
// A tile gives each lane four 16-byte chunks, 1 KiB apart.  Transposed so that byte lane s
// of register r_t holds byte t of chunk s, the byte before every byte of r_t is the same
// byte lane of r_{t-1}: prev1 is the previous register itself, and the nibble indices and
// sign masks of prev1 are those computed for r_{t-1} one step earlier, with no byte
// alignment at all.

// 4x4 byte transpose: r_k = byte k of a, b, c, d (in byte lanes 0..3).
__device__ __forceinline__ void transpose4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t& r0,
                                           uint32_t& r1, uint32_t& r2, uint32_t& r3) {
  const uint32_t t0 = perm(b, a, 0x05010400u);  // a0 b0 a1 b1
  const uint32_t t1 = perm(d, c, 0x05010400u);  // c0 d0 c1 d1
  const uint32_t t2 = perm(b, a, 0x07030602u);  // a2 b2 a3 b3
  const uint32_t t3 = perm(d, c, 0x07030602u);  // c2 d2 c3 d3
  r0 = perm(t1, t0, 0x05040100u);
  r1 = perm(t1, t0, 0x07060302u);
  r2 = perm(t3, t2, 0x05040100u);
  r3 = perm(t3, t2, 0x07060302u);
}

// The same transposition by another route: rows 0-1 and 2-3 are first gathered from
// chunks a, c and b, d.  (The comparison form below uses it, so that the compiler keeps
// the two forms' registers apart instead of holding one transposition for both.)
__device__ __forceinline__ void transpose4b(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t& r0,
                                            uint32_t& r1, uint32_t& r2, uint32_t& r3) {
  const uint32_t x01 = perm(c, a, 0x05040100u);  // a0 a1 c0 c1
  const uint32_t y01 = perm(d, b, 0x05040100u);  // b0 b1 d0 d1
  const uint32_t x23 = perm(c, a, 0x07060302u);  // a2 a3 c2 c3
  const uint32_t y23 = perm(d, b, 0x07060302u);  // b2 b3 d2 d3
  r0 = perm(y01, x01, 0x06020400u);
  r1 = perm(y01, x01, 0x07030501u);
  r2 = perm(y23, x23, 0x06020400u);
  r3 = perm(y23, x23, 0x07030501u);
}

// Values of the register before the current one (prev1), and must23's inputs.
struct LaneCarry {
  uint32_t neg, sh, sl, half;  // of r_{t-1}: sign mask, high-nibble and low-nibble indices, half selector
  uint32_t f;                  // bit 7: r_{t-1} >= 0xF0
  uint32_t g1, g2;             // g of r_{t-1} and r_{t-2} (bit 7: the byte >= 0xE0 or the byte before >= 0xF0)
};

__device__ __forceinline__ uint32_t sign_mask(uint32_t r) { return perm(r, r << 8, kSignSel); }

// Carried values for a run that starts after the registers q1, q2, q3 (bytes t-3, t-2, t-1).
__device__ __forceinline__ LaneCarry lanes_halo(uint32_t q1, uint32_t q2, uint32_t q3) {
  LaneCarry c;
  c.neg = sign_mask(q3);
  c.sh = (q3 >> 4) & 0x07070707u;
  c.sl = q3 & 0x07070707u;
  c.half = low_half_selector(q3);
  c.f = ge_mask7(q3, 0x10101010u);
  c.g1 = or_and(ge_mask7(q3, 0x20202020u), ge_mask7(q2, 0x10101010u), 0x80808080u);
  c.g2 = or_and(ge_mask7(q2, 0x20202020u), ge_mask7(q1, 0x10101010u), 0x80808080u);
  return c;
}

// 4x4 byte transpose (as transpose4) that also gives the sign masks of rows 0 and 2: the
// first step gathers each pair of rows with row 0 (2) in the odd bytes, where
// v_perm_b32's sign selectors read it.
__device__ __forceinline__ void transpose4s(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t& r0,
                                            uint32_t& r1, uint32_t& r2, uint32_t& r3, uint32_t& n0, uint32_t& n2) {
  const uint32_t x10 = perm(c, a, 0x04050001u);  // a1 a0 c1 c0
  const uint32_t y10 = perm(d, b, 0x04050001u);  // b1 b0 d1 d0
  const uint32_t x32 = perm(c, a, 0x06070203u);  // a3 a2 c3 c2
  const uint32_t y32 = perm(d, b, 0x06070203u);  // b3 b2 d3 d2
  r0 = perm(y10, x10, 0x07030501u);
  r1 = perm(y10, x10, 0x06020400u);
  r2 = perm(y32, x32, 0x07030501u);
  r3 = perm(y32, x32, 0x06020400u);
  n0 = perm(y10, x10, kSignSel);
  n2 = perm(y32, x32, kSignSel);
}

// Errors of register r (sections 6.1-6.2) with sign mask neg, ORed into acc; c moves on to r.
__device__ __forceinline__ uint32_t lanes_step(uint32_t acc, uint32_t r, uint32_t neg, LaneCarry& c) {
  const uint32_t sh = (r >> 4) & 0x07070707u;
  const uint32_t sc = lookup3(c.sh, c.sl, sh, c.neg, neg, c.half);
  const uint32_t g = or_and(ge_mask7(r, 0x20202020u), c.f, 0x80808080u);
  acc = or_xor(acc, sc, c.g2);  // must23 at t is g of t-2
  c.g2 = c.g1;
  c.g1 = g;
  c.f = ge_mask7(r, 0x10101010u);
  c.neg = neg;
  c.sh = sh;
  c.sl = r & 0x07070707u;
  c.half = low_half_selector(r);
  return acc;
}

// Errors of the four 16-byte chunks x0..x3 (each preceded by the dword p0..p3), ORed into
// acc: the same decision as chunk_errors on each chunk.  With PROBE, bit 7 of the bytes of
// *f_seen is also set where a byte of the chunks is >= 0xF0.
template <bool PROBE = false, class V>
__device__ __forceinline__ uint32_t chunks4_errors(uint32_t acc, const V& x0, const V& x1, const V& x2, const V& x3,
                                                   uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3,
                                                   uint32_t* f_seen = nullptr) {
  uint32_t q0, q1, q2, q3;
  transpose4(p0, p1, p2, p3, q0, q1, q2, q3);
  LaneCarry c = lanes_halo(q1, q2, q3);
  const uint32_t w[4][4] = {{x0.x, x1.x, x2.x, x3.x}, {x0.y, x1.y, x2.y, x3.y},
                            {x0.z, x1.z, x2.z, x3.z}, {x0.w, x1.w, x2.w, x3.w}};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t r0, r1, r2, r3, n0, n2;
    transpose4s(w[j][0], w[j][1], w[j][2], w[j][3], r0, r1, r2, r3, n0, n2);
    acc = lanes_step(acc, r0, n0, c);
    if (PROBE) *f_seen |= c.f;
    acc = lanes_step(acc, r1, sign_mask(r1), c);
    if (PROBE) *f_seen |= c.f;
    acc = lanes_step(acc, r2, n2, c);
    if (PROBE) *f_seen |= c.f;
    acc = lanes_step(acc, r3, sign_mask(r3), c);
    if (PROBE) *f_seen |= c.f;
  }
  return acc;
}

// ---- text without bytes >= 0xF0, across the byte lanes ---------------------------------------
// Where no byte of a position's window (its byte c and the three before it, p1 p2 p3) is
// >= 0xF0, must23 (6.2) is M = p2 >= 0xE0 and the table product of 6.1 is non-zero for: a
// lead p1 before a byte that is not a continuation (too short), an ASCII p1 before a
// continuation (too long), a continuation after C0 or C1 (overlong 2), after E0 below A0
// (overlong 3) and after ED from A0 on (surrogate); bit 7 is two continuations in a row.
// With K = "c is a continuation" and N = "p1 >= 0xC0, or M" (c must be a continuation),
// this form flags a position iff
//   K != N, or K and (p1 is C0/C1, or p1 is ED and c >= A0, or p1 is E0 and c < A0).
// The checks of 6.1-6.2 flag exactly these positions and, besides, a continuation after an
// ASCII or lead p1 where M holds; there the position before is flagged by both (p1 is not
// a continuation, and the byte before it is a lead >= 0xE0), so the first flagged position
// of any text is the same.  Every comparison is bit 7 of v_lerp_u8: a position costs eight
// comparisons and seven three-input logic operations, against nineteen operations in the
// table form.
//
// To know that no byte >= 0xF0 was there, a byte >= 0xF0 as p1 flags the position after
// it (it joins the C0/C1 case), and the two bytes before a run are tested on their own.
// A run that comes out without any flag therefore had no such byte in any window and no
// first flag of the checks (a flag of theirs that this form leaves out follows a flag of
// both, at the last byte of the run before at the latest); otherwise the caller checks it
// again with the table form.

struct ThreeCarry {
  uint32_t l1;    // r_{t-1} >= 0xC0
  uint32_t e1;    // r_{t-1} >= 0xE0 (M two positions on)
  uint32_t m;     // r_{t-2} >= 0xE0: M of this position
  uint32_t u, v;  // r_{t-1} is C0, C1 or >= 0xF0, or (u) ED, or (v) E0
};

__device__ __forceinline__ void three_lead(uint32_t r, uint32_t l, uint32_t e, uint32_t& u, uint32_t& v) {
  const uint32_t p = UTF8V_BITOP3(l, ge_mask7(r, 0x3E3E3E3Eu), ge_mask7(r, 0x10101010u), (a & ~b) | c);
  u = UTF8V_BITOP3(p, ge_mask7(r, 0x13131313u), ge_mask7(r, 0x12121212u), a | (b & ~c));  // ... or ED
  v = UTF8V_BITOP3(p, e, ge_mask7(r, 0x1F1F1F1Fu), a | (b & ~c));                          // ... or E0
}

// Carried values for a run after the registers q1, q2, q3 (bytes t-3, t-2, t-1); a byte
// >= 0xF0 in q1 or q2 is flagged in acc.
__device__ __forceinline__ ThreeCarry three_halo(uint32_t q1, uint32_t q2, uint32_t q3, uint32_t& acc) {
  ThreeCarry c;
  c.l1 = ge_mask7(q3, 0x40404040u);
  c.e1 = ge_mask7(q3, 0x20202020u);
  c.m = ge_mask7(q2, 0x20202020u);
  three_lead(q3, c.l1, c.e1, c.u, c.v);
  acc = UTF8V_BITOP3(acc, ge_mask7(q1, 0x10101010u), ge_mask7(q2, 0x10101010u), a | b | c);
  return c;
}

// Flags of register r (bit 7 of each byte) ORed into acc; c moves on to r.
__device__ __forceinline__ uint32_t three_step(uint32_t acc, uint32_t r, ThreeCarry& c) {
  const uint32_t l = ge_mask7(r, 0x40404040u);
  const uint32_t e = ge_mask7(r, 0x20202020u);
  const uint32_t k = UTF8V_BITOP3(r, l, 0u, a & ~b);                   // continuation
  const uint32_t x = UTF8V_BITOP3(c.l1, c.m, k, (a | b) ^ c);          // K != N
  const uint32_t s = select_bits(ge_mask7(r, 0x60606060u), c.u, c.v);  // c >= A0 ? (.., ED) : (.., E0)
  acc = UTF8V_BITOP3(acc, x, s, a | b | c);
  c.m = c.e1;
  c.e1 = e;
  c.l1 = l;
  three_lead(r, l, e, c.u, c.v);
  return acc;
}

// The four 16-byte chunks x0..x3 (each preceded by the dword p0..p3) in the form above:
// bit 7 of a byte of the result is set where a position is flagged or a byte >= 0xF0
// was seen (other bits are left over from the comparisons).
template <class V>
__device__ __forceinline__ uint32_t chunks4_three(uint32_t acc, const V& x0, const V& x1, const V& x2, const V& x3,
                                                  uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3) {
  uint32_t q0, q1, q2, q3;
  transpose4b(p0, p1, p2, p3, q0, q1, q2, q3);
  ThreeCarry c = three_halo(q1, q2, q3, acc);
  const uint32_t w[4][4] = {{x0.x, x1.x, x2.x, x3.x}, {x0.y, x1.y, x2.y, x3.y},
                            {x0.z, x1.z, x2.z, x3.z}, {x0.w, x1.w, x2.w, x3.w}};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint32_t r0, r1, r2, r3;
    transpose4b(w[j][0], w[j][1], w[j][2], w[j][3], r0, r1, r2, r3);
    acc = three_step(acc, r0, c);
    acc = three_step(acc, r1, c);
    acc = three_step(acc, r2, c);
    acc = three_step(acc, r3, c);
  }
  return acc;
}

// ---- per-string masking (CSR batches) ----------------------------------------------------
// s / sp: string-start masks (0xFF at positions where a string starts) of x and of the
// dword before it.  Bytes of an earlier string count as zero (section 6: the stream
// starts after zeros), so at a start prev1 is zero, must23 ignores bytes before the
// start, and the string that ends at a start position gets the end check of 6.3.
// gq at byte j: bit 7 = b[j] >= 0xE0, or b[j-1] >= 0xF0 when j is not a start.

struct MaskedCarry {
  uint32_t neg2, sh2, gq;
};

// Carried values of the dword p before a run (only its top bytes are used).
__device__ __forceinline__ MaskedCarry masked_halo(uint32_t p, uint32_t sp) {
  MaskedCarry c;
  c.neg2 = perm(p, p, kSignSel);
  c.sh2 = (p >> 4) & 0x07070707u;
  // a | (b & ~c)
  c.gq = or_andn(ge_mask7(p, 0x20202020u), ge_mask7(p << 8, 0x10101010u), sp);
  return c;
}

// One dword x (string-start mask s) after xp (mask sp): regular errors ORed into acc,
// end-check errors ORed into tail.
__device__ __forceinline__ void masked_next(uint32_t x, uint32_t xp, uint32_t s, uint32_t sp, MaskedCarry& c,
                                            uint32_t& acc, uint32_t& tail) {
  const uint32_t prev1 = align(x, xp, 3);
  const uint32_t s1 = align(s, sp, 3);                    // position i-1 starts a string
  const uint32_t neg2 = perm(x, prev1, kSignSel);
  const uint32_t sh2 = (x >> 4) & 0x07070707u;
  const uint32_t gq = or_andn(ge_mask7(x, 0x20202020u), ge_mask7(prev1, 0x10101010u), s);
  // prev1 of another string acts as zero: byte_1_high then reads 0x02 (neg1 cleared)
  const uint32_t neg1 = align(neg2, c.neg2, 3) & ~s;
  const uint32_t sc = lookup3(align(sh2, c.sh2, 3), prev1 & 0x07070707u, sh2, neg1, neg2, low_half_selector(prev1));
  const uint32_t m = align(gq, c.gq, 2);                  // bit 7: must23 before the string masks
  // must23 needs the bytes i-2 (i-3) in the string of i: no start at i, i-1 (i-2 is in gq)
  const uint32_t m23 = andn_and(m, s | s1, 0x80808080u);
  // end check of the string holding byte i-1, at a start position i
  const uint32_t u = or_andn(ge_mask7(prev1, 0x40404040u), m, s1);
  tail |= and3(u, s, 0x80808080u);
  acc = or_xor(acc, sc, m23);
  c.neg2 = neg2;
  c.sh2 = sh2;
  c.gq = gq;
}

// Index (0..3) of the lowest non-zero byte of a non-zero register.
__device__ __forceinline__ int first_byte(uint32_t e) { return __builtin_ctz(e) >> 3; }

}  // namespace utf8v

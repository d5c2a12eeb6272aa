// Morton (Z-order) indexing of the uniform quadtree: x in the even bits, y in the odd
// bits.  The four children of cell k at level l are 4k + q at level l + 1 with
// q = (child x bit) | (child y bit) << 1, so siblings are adjacent and a cell's parity
// class is k & 3.  Plain constexpr functions: host C++ and device code (HIP treats
// constexpr functions as usable on both sides) share them.
#pragma once

#include <cstdint>

namespace fmm {

constexpr uint32_t spread_bits(uint32_t v)
{
    v &= 0x0000ffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

constexpr uint32_t gather_bits(uint32_t v)
{
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0f0f0f0fu;
    v = (v | (v >> 4)) & 0x00ff00ffu;
    v = (v | (v >> 8)) & 0x0000ffffu;
    return v;
}

constexpr uint32_t morton_encode(uint32_t x, uint32_t y) { return spread_bits(x) | (spread_bits(y) << 1); }
constexpr uint32_t morton_x(uint32_t m) { return gather_bits(m); }
constexpr uint32_t morton_y(uint32_t m) { return gather_bits(m >> 1); }

// First global cell index of level l when all levels are stored back to back:
// sum_{k<l} 4^k = (4^l - 1)/3.
constexpr int64_t level_base(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }

}  // namespace fmm

// Morton (Z-order) key of a site, shared by the dataset ordering and the batched ordering:
// each coordinate clamped to [0, 1] and quantised to 16 bits, q = min(floor(c * 2^16), 2^16 - 1);
// the bits of q_x go to the even positions and those of q_y to the odd positions of a 32-bit
// key; (longitude, latitude) sites in degrees are first mapped to ((lon + 180) / 360,
// (lat + 90) / 180).
#pragma once
#include "common.h"

namespace mpgeo {

namespace {

__device__ inline uint32_t spread_bits(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t quantise(double c) {
    c = c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c);
    const double q = floor(c * 65536.0);
    return q > 65535.0 ? 65535u : (uint32_t)q;
}

__device__ inline uint32_t morton_key(double x, double y, int lonlat) {
    if (lonlat) {
        x = (x + 180.0) / 360.0;
        y = (y + 90.0) / 180.0;
    }
    return spread_bits(quantise(x)) | (spread_bits(quantise(y)) << 1);
}

}  // namespace

}  // namespace mpgeo

// Tile windows and patches of the mass apply, shared by the kernels that
// write the patches and those that read them.
//
// A mass apply on a tile of TILE^3 elements produces the contributions to the
// basis functions whose support meets the tile: per component a window of
// (TILE + K - 1) functions along each axis, K the number of functions of that
// axis' tag nonzero on one element.  Windows of neighbouring tiles overlap;
// each tile writes its window as a "patch" and a reader sums, in a fixed
// order, the (at most eight) patches that cover an output.
#pragma once

#include "kmx_internal.hpp"

namespace kmx {

template <int P, int SPACE, int C>
struct Lay {  // window layout of component C of a form space inside one tile
    static constexpr int tx = space_tag(SPACE, C, 0), ty = space_tag(SPACE, C, 1), tz = space_tag(SPACE, C, 2);
    static constexpr int Kx = tag_support(P, tx), Ky = tag_support(P, ty), Kz = tag_support(P, tz);
    static constexpr int Wx = TILE + Kx - 1, Wy = TILE + Ky - 1, Wz = TILE + Kz - 1;
    static constexpr int plane = Wx * Wy;
    static constexpr int size = plane * Wz;
};

// Patch layout of one component: [tz][ty][lz][ly][tx][lx], the x rows of the
// tiles along x side by side, so that a row of outputs gathers from
// contiguous memory.  One component's patches hold nt^3 Wx Wy Wz entries
// (N <= 72 elements per axis: nt <= 18, windows <= 8 per axis), far below
// 2^31, so offsets inside a component are 32-bit.
template <class L>
__host__ __device__ inline int patch_row(int nt, int ty, int tz, int ly, int lz) {
    return (((tz * nt + ty) * L::Wz + lz) * L::Wy + ly) * nt * L::Wx;
}

template <class L>
__host__ __device__ inline int64_t patch_at(int nt, int tx, int ty, int tz, int lx, int ly, int lz) {
    return patch_row<L>(nt, ty, tz, ly, lz) + tx * L::Wx + lx;
}

// Patch gather: the sum of the tile patches covering basis function (gx, gy,
// gz) of component C, in a fixed order (tiles by increasing z, y, x).
template <int P, int SPACE, int C>
__device__ inline double gather_one(const double* __restrict__ patch, int nt, int gz, int gy, int gx) {
    using L = Lay<P, SPACE, C>;
    const int rx = gx - tag_offset(L::tx), ry = gy - tag_offset(L::ty), rz = gz - tag_offset(L::tz);
    int hx = rx / TILE, hy = ry / TILE, hz = rz / TILE;
    hx = hx > nt - 1 ? nt - 1 : hx;
    hy = hy > nt - 1 ? nt - 1 : hy;
    hz = hz > nt - 1 ? nt - 1 : hz;
    // the candidate tiles h - 1 and h per axis, in a fixed order; a candidate
    // that does not cover the entry contributes zero and is not read (the
    // lanes whose candidate covers it read, the others are masked off)
    bool vx[2], vy[2], vz[2];
    int tx[2], ty[2], tz[2], lx[2], ly[2], lz[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
        const int ax = hx - 1 + d, ay = hy - 1 + d, az = hz - 1 + d;
        vx[d] = ax >= 0 && rx - ax * TILE < L::Wx;
        vy[d] = ay >= 0 && ry - ay * TILE < L::Wy;
        vz[d] = az >= 0 && rz - az * TILE < L::Wz;
        tx[d] = vx[d] ? ax : hx;
        ty[d] = vy[d] ? ay : hy;
        tz[d] = vz[d] ? az : hz;
        lx[d] = vx[d] ? rx - tx[d] * TILE : 0;
        ly[d] = vy[d] ? ry - ty[d] * TILE : 0;
        lz[d] = vz[d] ? rz - tz[d] * TILE : 0;
    }
    // the four (z, y) row offsets and the two x offsets, then the reads
    int row[4], col[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) row[k] = patch_row<L>(nt, ty[k & 1], tz[k >> 1], ly[k & 1], lz[k >> 1]);
#pragma unroll
    for (int d = 0; d < 2; ++d) col[d] = tx[d] * L::Wx + lx[d];
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int dz = k >> 2, dy = (k >> 1) & 1, dx = k & 1;
        v[k] = 0.0;
        if (vz[dz] && vy[dy] && vx[dx]) v[k] = patch[row[k >> 1] + col[k & 1]];
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    return s;
}

}  // namespace kmx

// lattice.hpp -- compile-time lattice descriptors for the GPU kernels.
//
// Velocity sets D2Q9, D3Q19, D3Q27 (paper Sec. 2, Fig. "lattice"; Sec. 3.2
// lattice class hierarchy).  Index 0 is the rest vector, 1..Q-1 follow the
// figure's order.  Weights are the standard ones by |c|^2 (the paper does not
// print them): D2Q9 4/9, 1/9, 1/36; D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27,
// 1/54, 1/216.
//
// Internal axes.  The kernels always see three axes (X, Y, Z) with Z the
// contiguous one.  A 3-D grid maps (x, y, z) -> (X, Y, Z).  A 2-D grid maps
// (x, y) -> (Y, Z) with a dummy X of length 1, so a D2Q9 vector (cx, cy) is
// stored here as (0, cx, cy).
#pragma once
#include <cstdint>

namespace lbm {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    // internal (X, Y, Z) components; external (cx, cy) = (Y, Z)
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0}, {0, 1, 0}, {0, 0, 1}, {0, -1, 0}, {0, 0, -1},
        {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};
    static constexpr double wn[4] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0, 0.0};
    static constexpr int den_t = 2;  // sum over a Zou-He unknown set of c_t^2
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
        {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
        {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
        {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};
    static constexpr double wn[4] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0, 0.0};
    static constexpr int den_t = 2;
};

struct D3Q27 {
    static constexpr int Q = 27;
    static constexpr int D = 3;
    static constexpr int8_t c[Q][3] = {
        {0, 0, 0},
        {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
        {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
        {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
        {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1},
        {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1},
        {-1, 1, 1}, {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}};
    static constexpr double wn[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
    static constexpr int den_t = 6;
};

template <class L>
__host__ __device__ constexpr int cnorm2(int i) {
    return L::c[i][0] * L::c[i][0] + L::c[i][1] * L::c[i][1] + L::c[i][2] * L::c[i][2];
}

template <class L>
__host__ __device__ constexpr double weight(int i) {
    return L::wn[cnorm2<L>(i)];
}

template <class L>
__host__ __device__ constexpr int opp(int i) {
    int r = 0;
    for (int j = 0; j < L::Q; ++j)
        if (L::c[j][0] == -L::c[i][0] && L::c[j][1] == -L::c[i][1] && L::c[j][2] == -L::c[i][2]) r = j;
    return r;
}

// Face bits of the internal box: bit 2a is the low face of axis a, bit 2a+1
// the high face.  The source x - c_i of population i lies across the low face
// of axis a when c_ia = +1 and the cell sits on that face.
template <class L>
__host__ __device__ constexpr uint32_t src_face_bits(int i) {
    uint32_t m = 0;
    for (int a = 0; a < 3; ++a) {
        if (L::c[i][a] > 0) m |= 1u << (2 * a);
        if (L::c[i][a] < 0) m |= 1u << (2 * a + 1);
    }
    return m;
}

// Faces any direction's source can cross (the lattice's axes).
template <class L>
__host__ __device__ constexpr uint32_t all_face_bits() {
    uint32_t m = 0;
    for (int i = 0; i < L::Q; ++i) m |= src_face_bits<L>(i);
    return m;
}

}  // namespace lbm

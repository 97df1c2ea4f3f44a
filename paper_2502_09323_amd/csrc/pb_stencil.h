// pb_stencil.h -- the 7-point operator read from the node-code map (device helpers shared by
// the build, the Jacobi and multigrid solvers and the refined-grid coefficients).
//
// An edge inside one medium has K = h*eps_in or h*eps_out; a cut edge reads its WHA value from
// the compact table ck[3*slot + axis] (paper Sect. 3.2, eq. WHA).  The edge along +axis from
// a node is described by that node's code.  The diagonal of a node is the sum of its six
// edge weights and its lumped ionic term (paper Sect. 3.1, eq. matrixequation), always summed
// in the order of diag_sum, so that every kernel that forms it gets the same bits.
#pragma once

#include "pb_internal.h"

namespace pbk {
namespace stencil {

// The table index of the edge along +axis from a node (slot 0 for an uncut edge): the table
// is always read and the result blended arithmetically (ck_blend), so that the load is never
// turned into a branch whose join would wait on every load in flight.
__device__ __forceinline__ int64_t ck_index(uint32_t c, int ax)
{
    return (c & (C_CUTX << ax)) ? 3 * (int64_t)(c >> C_SLOT_SHIFT) + ax : 0;
}

// v (the table value) for a cut edge, else h*eps of the node's medium; m is 0 or 1, so the
// blend returns one of the two exactly
template <typename T>
__device__ __forceinline__ T ck_blend(T v, uint32_t c, int ax, T kin, T kout)
{
    const T base = (c & C_SOLUTE) ? kin : kout;
    const T m = (c & (C_CUTX << ax)) ? (T)1 : (T)0;
    return v * m + base * ((T)1 - m);
}

template <typename T>
__device__ __forceinline__ T edgeK(uint32_t c, int ax, const T* __restrict__ ck, T kin, T kout)
{
    return ck_blend(ck[ck_index(c, ax)], c, ax, kin, kout);
}

// the diagonal from the six edge weights (x-, x+, y-, y+, z-, z+) and the ionic term
template <typename T>
__device__ __forceinline__ T diag_sum(T kxm, T kxp, T kym, T kyp, T kzm, T kzp, T mt)
{
    return ((kxm + kxp) + (kym + kyp)) + ((kzm + kzp) + mt);
}

// the six edge weights of node e (x-, x+, y-, y+, z-, z+) and its ionic term
template <typename T>
struct NodeK {
    T xm, xp, ym, yp, zm, zp, m;
    __device__ __forceinline__ T diag() const { return diag_sum(xm, xp, ym, yp, zm, zp, m); }
};

template <typename T>
__device__ __forceinline__ NodeK<T> node_k(const Grid& g, const uint32_t* __restrict__ code,
                                           const T* __restrict__ ck, T kin, T kout, T mass, int64_t e)
{
    const int64_t sx = (int64_t)g.ny * g.S, sy = g.S;
    const uint32_t c = code[e];
    NodeK<T> k;
    k.xm = edgeK(code[e - sx], 0, ck, kin, kout);
    k.xp = edgeK(c, 0, ck, kin, kout);
    k.ym = edgeK(code[e - sy], 1, ck, kin, kout);
    k.yp = edgeK(c, 1, ck, kin, kout);
    k.zm = edgeK(code[e - 1], 2, ck, kin, kout);
    k.zp = edgeK(c, 2, ck, kin, kout);
    k.m = (c & C_SOLUTE) ? (T)0 : mass;
    return k;
}

template <typename T>
__device__ __forceinline__ T node_diag(const Grid& g, const uint32_t* __restrict__ code, const T* __restrict__ ck,
                                       T kin, T kout, T mass, int64_t e)
{
    return node_k(g, code, ck, kin, kout, mass, e).diag();
}

}  // namespace stencil
}  // namespace pbk

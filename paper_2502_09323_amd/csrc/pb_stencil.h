// pb_stencil.h -- the 7-point operator read from the node-code map (device helpers).
//
// An edge inside one medium has K = h*eps_in or h*eps_out; a cut edge reads its WHA value from
// the compact table ck[3*slot + axis] (paper Sect. 3.2, eq. WHA).  The edge along +axis from
// a node is described by that node's code.  The diagonal of a node is the sum of its six
// edge weights and its lumped ionic term (paper Sect. 3.1, eq. matrixequation).
#pragma once

#include "pb_internal.h"

namespace pbk {
namespace stencil {

// The table is read for every edge (entry 0 for an uncut one) and the result blended
// arithmetically, so that no load sits behind a branch.
template <typename T>
__device__ __forceinline__ T edgeK(uint32_t c, int ax, const T* __restrict__ ck, T kin, T kout)
{
    const bool cut = (c & (C_CUTX << ax)) != 0;
    const T v = ck[cut ? 3 * (int64_t)(c >> C_SLOT_SHIFT) + ax : 0];
    const T base = (c & C_SOLUTE) ? kin : kout;
    const T m = cut ? (T)1 : (T)0;
    return v * m + base * ((T)1 - m);
}

// the six edge weights of node e (x-, x+, y-, y+, z-, z+) and its ionic term
template <typename T>
struct NodeK {
    T xm, xp, ym, yp, zm, zp, m;
    __device__ __forceinline__ T diag() const { return ((xm + xp) + (ym + yp)) + ((zm + zp) + m); }
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

}  // namespace stencil
}  // namespace pbk

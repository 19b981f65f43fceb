// se_device.h -- device helpers shared by the library's kernels.
#pragma once

#include "se_internal.h"

// Grid coordinate u = (x - x0)/h (IEEE division, FP64) of one axis.
__device__ __forceinline__ double se_gridcoord(const se_grid_geom& g, int d, double x)
{
    return (x - g.x0[d]) / g.h[d];
}

// Grid anchor floor((x - x0)/h), clamped to the grid (Sec. 3.3: the window
// support of a point spans anchor - P/2 + 1 .. anchor + P/2).
__device__ __forceinline__ int se_anchor(const se_grid_geom& g, int d, double x)
{
    double u = se_gridcoord(g, d, x);
    int a = (int)floor(u);
    if (a < 0) a = 0;
    if (a > g.Mg[d] - 1) a = g.Mg[d] - 1;
    return a;
}

__device__ __forceinline__ int se_floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// PKB weight of stencil offset q at local coordinate s in [0,1] within the
// subinterval: Horner in sigma = 2 s - 1 over coef[q][0..nu].
template <typename R>
__device__ __forceinline__ R se_pkb_eval(const double* coef, int nu, int q, R s)
{
    const double* c = coef + q * (nu + 1);
    R sig = (R)2 * s - (R)1;
    R acc = (R)c[nu];
    for (int k = nu - 1; k >= 0; k--) acc = acc * sig + (R)c[k];
    return acc;
}

__device__ __forceinline__ double se_readlane(double v, int lane)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_readlane(lo, lane);
    hi = __builtin_amdgcn_readlane(hi, lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float se_readlane(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the hardware block id so that every XCD works on one contiguous
// range of logical blocks (spatial neighbours share an L2).  Bijective on
// [0, nblocks).
__device__ __forceinline__ int se_xcd_block(int b, int nblocks)
{
    const int q = nblocks / 8, r = nblocks % 8;
    const int xcd = b % 8, idx = b / 8;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename R>
struct se_cplx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ se_cplx<R> cmul(se_cplx<R> a, se_cplx<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

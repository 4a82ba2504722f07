// Halo buffer layout of the virtual split (used by halo.hip).
//
// Buffer: subdomains s = a + Pi*(b + Pj*c) in order; per subdomain its faces
// -x, +x, -y, +y, -z, +z that are cuts (not cavity walls); per face the
// fields p, u, v, w, T with width > 0; per field the box of the w interior
// layers next to the face over the subdomain's tangential extent, in
// (k, j, i) order, i fastest (Sec. 4.5, Listings 1-2).
#pragma once

#include "cavity_internal.h"

namespace cav {

// Cut faces along one axis among the first m of P subdomains.
__device__ __forceinline__ long long cuts_before(int P, int m)
{
    return m == 0 ? 0 : (long long)(m - 1) + min(m, P - 1);
}
__device__ __forceinline__ int cuts_of(int P, int a)
{
    return (a > 0 ? 1 : 0) + (a < P - 1 ? 1 : 0);
}

// Whether `face` of subdomain (a, b, c) is a cavity wall.
__device__ __forceinline__ bool face_is_wall(const HaloGeom& h, int a, int b, int c, int face)
{
    const int ax = face >> 1;
    const int coord = ax == 0 ? a : (ax == 1 ? b : c);
    return (face & 1) ? coord == h.P[ax] - 1 : coord == 0;
}

// Offset, in tangential cells, of the segment of `face` of subdomain
// (a, b, c): the cut faces of all earlier subdomains (closed form), then the
// earlier cut faces of this one.  Multiply by wsum for the element offset.
__device__ __forceinline__ long long face_offset(const HaloGeom& h, int a, int b, int c, int face)
{
    const int Pi = h.P[0], Pj = h.P[1], Pk = h.P[2];
    const long long Ax = h.area[0], Ay = h.area[1], Az = h.area[2];
    long long u = (long long)c * (Ax * 2LL * (Pi - 1) * Pj + Ay * 2LL * (Pj - 1) * Pi)
                + Az * cuts_before(Pk, c) * Pi * Pj
                + (long long)b * Ax * 2LL * (Pi - 1) + Ay * cuts_before(Pj, b) * Pi
                + Az * cuts_of(Pk, c) * (long long)Pi * b
                + Ax * cuts_before(Pi, a) + Ay * cuts_of(Pj, b) * (long long)a
                + Az * cuts_of(Pk, c) * (long long)a;
    for (int f2 = 0; f2 < face; ++f2)
        if (!face_is_wall(h, a, b, c, f2)) u += h.area[f2 >> 1];
    return u;
}

}  // namespace cav

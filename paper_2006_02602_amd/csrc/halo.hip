// In-device halo pack / unpack for gfx950 (Xue & Roy, arXiv:2006.02602,
// Sec. 4.5: "Optimized V1" packs the noncontiguous i faces into a contiguous
// buffer in parallel on the device, "V2" sends each field with its own
// stencil width, "V3" extends the buffers to the j and k faces).
//
// One launch covers every (subdomain, face) pair of the virtual split:
// blockIdx.y = subdomain * 6 + face, blockIdx.x walks the face's tangential
// cells.  Each thread owns one tangential cell of the face and moves all
// fields and layers of it, so the buffer position needs one integer
// division per thread.  The buffer layout is in halo_layout.h.
#include "cavity_internal.h"
#include "halo_layout.h"

namespace cav {

template <typename Real, bool PACK>
__global__ __launch_bounds__(256) void halo_kernel(Dims d, HaloGeom h, StateT<Real> q, Real* buf)
{
    const int slot = blockIdx.y;
    const int s = slot / 6, face = slot - 6 * s;
    const int Pi = h.P[0], Pj = h.P[1];
    const int a = s % Pi, c = s / (Pi * Pj), b = (s / Pi) % Pj;
    const int axis = face >> 1;
    const bool high = face & 1;
    const int coord = axis == 0 ? a : (axis == 1 ? b : c);
    if (high ? coord == h.P[axis] - 1 : coord == 0) return;     // a cavity wall, not a cut

    const int area = (int)h.area[axis];
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= area) return;

    // offset (in tangential cells) of this face's segment
    const long long u = face_offset(h, a, b, c, face);
    Real* __restrict__ B = buf + u * h.wsum;

    // this thread's tangential cell, the first layer's offset per field and
    // the stride between layers (all fields first, then all stores, so that
    // every load is in flight before the first store)
    const int ex = h.e[0], ey = h.e[1], ez = h.e[2];
    int ta, tb;                       // tangential coordinates
    long long lay_b;                  // buffer stride between layers
    int lay_q;                        // state stride between layers
    if (axis == 0) { ta = t % ey; tb = t / ey; lay_b = 1; lay_q = 1; }
    else if (axis == 1) { ta = t % ex; tb = t / ex; lay_b = ex; lay_q = d.sy; }
    else { ta = t % ex; tb = t / ex; lay_b = (long long)ex * ey; lay_q = d.sz; }
    int qo[NF];
    long long bo[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int w = h.w[f];
        const long long base = (long long)h.wpre[f] * area;
        if (axis == 0) {
            const int gi = high ? (a + 1) * ex - w : a * ex;
            qo[f] = cell_off(d, gi, b * ey + ta, c * ez + tb);
            bo[f] = base + (long long)t * w;
        } else if (axis == 1) {
            const int gj = high ? (b + 1) * ey - w : b * ey;
            qo[f] = cell_off(d, a * ex + ta, gj, c * ez + tb);
            bo[f] = base + (long long)tb * w * ex + ta;
        } else {
            const int gk = high ? (c + 1) * ez - w : c * ez;
            qo[f] = cell_off(d, a * ex + ta, b * ey + tb, gk);
            bo[f] = base + (long long)tb * ex + ta;
        }
    }
    Real v0[NF], v1[NF];
    if (PACK) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const Real* __restrict__ Q = q.f[f];
            if (h.w[f] > 0) v0[f] = Q[qo[f]];
            if (h.w[f] > 1) v1[f] = Q[qo[f] + lay_q];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (h.w[f] > 0) B[bo[f]] = v0[f];
            if (h.w[f] > 1) B[bo[f] + lay_b] = v1[f];
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (h.w[f] > 0) v0[f] = B[bo[f]];
            if (h.w[f] > 1) v1[f] = B[bo[f] + lay_b];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Real* __restrict__ Q = q.f[f];
            if (h.w[f] > 0) Q[qo[f]] = v0[f];
            if (h.w[f] > 1) Q[qo[f] + lay_q] = v1[f];
        }
    }
}

template <typename Real>
hipError_t launch_halo(const Dims& d, const HaloGeom& h, StateT<Real> q, Real* buf, bool pack, hipStream_t s)
{
    const int nsub = h.P[0] * h.P[1] * h.P[2];
    dim3 grid(h.face_blocks, nsub * 6), block(256);
    if (pack)
        halo_kernel<Real, true><<<grid, block, 0, s>>>(d, h, q, buf);
    else
        halo_kernel<Real, false><<<grid, block, 0, s>>>(d, h, q, buf);
    return hipGetLastError();
}
template hipError_t launch_halo<double>(const Dims&, const HaloGeom&, StateT<double>, double*, bool, hipStream_t);
template hipError_t launch_halo<float>(const Dims&, const HaloGeom&, StateT<float>, float*, bool, hipStream_t);

}  // namespace cav

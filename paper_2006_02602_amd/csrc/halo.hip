// In-device halo pack / unpack for gfx950 (Xue & Roy, arXiv:2006.02602,
// Sec. 4.5: "Optimized V1" packs the noncontiguous i faces into a contiguous
// buffer in parallel on the device, "V2" sends each field with its own
// stencil width, "V3" extends the buffers to the j and k faces).
//
// One launch covers every cut face of the virtual split and nothing else:
// the grid is three ranges of blocks, one per axis, each (cut faces normal
// to that axis) x (blocks per face, sized to that axis' face area).  A
// thread moves HALO_ROWS tangential cells of one face, 256 cells apart, with
// all fields and layers of each: every load of the thread is in flight
// before its first store.  On j and k faces the lanes run along i, so loads
// and stores are coalesced rows.  On i faces a lane's layers are adjacent
// in memory (one 16-byte access for two FP64 layers when aligned) and
// consecutive lanes take consecutive rows, whose buffer entries are
// adjacent: the buffer side is coalesced, the state side moves one short
// run per row.  The buffer layout is in halo_layout.h.
#include "cavity_internal.h"
#include "halo_layout.h"

namespace cav {

template <typename Real>
struct Pair;
template <>
struct Pair<double> {
    using T = double2;
};
template <>
struct Pair<float> {
    using T = float2;
};

// Face `fidx` of the cut faces normal to `axis`: cut m (between subdomain
// coordinates m and m+1 along the axis), transverse subdomain pair tr, and
// side 0 = the +axis face of the lower subdomain, 1 = the -axis face of the
// upper one.
__device__ __forceinline__ void face_of(const HaloGeom& h, int axis, int fidx, int& a, int& b, int& c, int& face)
{
    const int side = fidx & 1, pair = fidx >> 1;
    const int cut = pair % (h.P[axis] - 1), tr = pair / (h.P[axis] - 1);
    const int m = cut + side;
    face = 2 * axis + (side ? 0 : 1);
    if (axis == 0) { a = m; b = tr % h.P[1]; c = tr / h.P[1]; }
    else if (axis == 1) { a = tr % h.P[0]; b = m; c = tr / h.P[0]; }
    else { a = tr % h.P[0]; b = tr / h.P[0]; c = m; }
}

template <typename Real, bool PACK>
__global__ __launch_bounds__(HALO_THREADS) void halo_kernel(Dims d, HaloGeom h, StateT<Real> q, Real* buf, int blk0)
{
    using R2 = typename Pair<Real>::T;
    int blk = blockIdx.x + blk0;
    const int axis = blk < h.blk_end[0] ? 0 : (blk < h.blk_end[1] ? 1 : 2);
    if (axis > 0) blk -= h.blk_end[axis - 1];
    const int fidx = blk / h.bpf[axis], fblk = blk - fidx * h.bpf[axis];
    int a, b, c, face;
    face_of(h, axis, fidx, a, b, c, face);
    const bool high = face & 1;
    const int area = (int)h.area[axis];

    // offset (in tangential cells) of this face's segment
    const long long u = face_offset(h, a, b, c, face);
    Real* __restrict__ B = buf + u * h.wsum;

    const int ex = h.e[0], ey = h.e[1], ez = h.e[2];
    // per field: state offset of the face's first layer at tangential cell
    // 0, and the buffer offset of its box
    int qbase[NF];
    long long bbase[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int w = h.w[f];
        bbase[f] = (long long)h.wpre[f] * area;
        if (axis == 0) qbase[f] = cell_off(d, high ? (a + 1) * ex - w : a * ex, b * ey, c * ez);
        else if (axis == 1) qbase[f] = cell_off(d, a * ex, high ? (b + 1) * ey - w : b * ey, c * ez);
        else qbase[f] = cell_off(d, a * ex, b * ey, high ? (c + 1) * ez - w : c * ez);
    }
    // this thread's tangential cells: (ta, tb) = (j, k) on i faces, (i, k)
    // on j faces, (i, j) on k faces, and their state offsets from qbase
    const int t0 = fblk * (HALO_THREADS * HALO_ROWS) + threadIdx.x;
    const int ne = axis == 0 ? ey : ex;
    int ta[HALO_ROWS], tb[HALO_ROWS], qo[HALO_ROWS];
    bool ok[HALO_ROWS];
#pragma unroll
    for (int r = 0; r < HALO_ROWS; ++r) {
        const int t = t0 + r * HALO_THREADS;
        ok[r] = t < area;
        ta[r] = t % ne;
        tb[r] = t / ne;
        qo[r] = axis == 0 ? tb[r] * d.sz + ta[r] * d.sy : (axis == 1 ? tb[r] * d.sz + ta[r] : tb[r] * d.sy + ta[r]);
    }
    // stride between layers in the state
    const int lay_q = axis == 0 ? 1 : (axis == 1 ? d.sy : d.sz);

    // buffer element of (tangential cell r, layer l) of field f: the box in
    // (k, j, i) order, i fastest
    auto bidx = [&](int f, int r, int l) -> long long {
        const int w = h.w[f];
        if (axis == 0) return bbase[f] + ((long long)tb[r] * ey + ta[r]) * w + l;
        if (axis == 1) return bbase[f] + ((long long)tb[r] * w + l) * ex + ta[r];
        return bbase[f] + (long long)l * area + (long long)tb[r] * ex + ta[r];
    };
    // two layers of an i face move as one pair where the address allows
    auto paired = [&](const Real* p) { return axis == 0 && (reinterpret_cast<uintptr_t>(p) % sizeof(R2)) == 0; };

    Real v[HALO_ROWS][NF][2];
    if (PACK) {
#pragma unroll
        for (int r = 0; r < HALO_ROWS; ++r) {
            if (!ok[r]) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const Real* __restrict__ Q = q.f[f] + qbase[f] + qo[r];
                const int w = h.w[f];
                if (w == 2 && paired(Q)) {
                    const R2 x = *reinterpret_cast<const R2*>(Q);
                    v[r][f][0] = x.x;
                    v[r][f][1] = x.y;
                } else {
                    if (w > 0) v[r][f][0] = Q[0];
                    if (w > 1) v[r][f][1] = Q[lay_q];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < HALO_ROWS; ++r) {
            if (!ok[r]) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int w = h.w[f];
                const long long o = bidx(f, r, 0);
                if (w == 2 && paired(B + o)) {
                    R2 x;
                    x.x = v[r][f][0];
                    x.y = v[r][f][1];
                    *reinterpret_cast<R2*>(B + o) = x;
                } else {
                    if (w > 0) B[o] = v[r][f][0];
                    if (w > 1) B[bidx(f, r, 1)] = v[r][f][1];
                }
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < HALO_ROWS; ++r) {
            if (!ok[r]) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const int w = h.w[f];
                const long long o = bidx(f, r, 0);
                if (w == 2 && paired(B + o)) {
                    const R2 x = *reinterpret_cast<const R2*>(B + o);
                    v[r][f][0] = x.x;
                    v[r][f][1] = x.y;
                } else {
                    if (w > 0) v[r][f][0] = B[o];
                    if (w > 1) v[r][f][1] = B[bidx(f, r, 1)];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < HALO_ROWS; ++r) {
            if (!ok[r]) continue;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                Real* __restrict__ Q = q.f[f] + qbase[f] + qo[r];
                const int w = h.w[f];
                if (w == 2 && paired(Q)) {
                    R2 x;
                    x.x = v[r][f][0];
                    x.y = v[r][f][1];
                    *reinterpret_cast<R2*>(Q) = x;
                } else {
                    if (w > 0) Q[0] = v[r][f][0];
                    if (w > 1) Q[lay_q] = v[r][f][1];
                }
            }
        }
    }
}

// first_axis 1 launches only the j- and k-face block ranges (the i faces
// were packed by the sweep's epilogue).
template <typename Real>
hipError_t launch_halo(const Dims& d, const HaloGeom& h, StateT<Real> q, Real* buf, bool pack, hipStream_t s,
                       int first_axis)
{
    const int blk0 = first_axis > 0 ? h.blk_end[first_axis - 1] : 0;
    const int nb = h.blk_end[2] - blk0;
    if (nb <= 0) return hipSuccess;
    if (pack)
        halo_kernel<Real, true><<<nb, HALO_THREADS, 0, s>>>(d, h, q, buf, blk0);
    else
        halo_kernel<Real, false><<<nb, HALO_THREADS, 0, s>>>(d, h, q, buf, blk0);
    return hipGetLastError();
}
template hipError_t launch_halo<double>(const Dims&, const HaloGeom&, StateT<double>, double*, bool, hipStream_t, int);
template hipError_t launch_halo<float>(const Dims&, const HaloGeom&, StateT<float>, float*, bool, hipStream_t, int);

}  // namespace cav

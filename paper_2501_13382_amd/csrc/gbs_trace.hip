// Ray-tracing stage on the device: the step before beam summation (paper
// Sec. 3.1: rays are traced through the environment first; Sec. 3.3: one
// thread per ray).  Writes the ray table the summation reads.
//
// Scene: the ground plane z = 0 (face 0) and axis-aligned boxes standing on
// it (walls -x, +x, -y, +y and a roof, each split into panels x panels
// cells).  Reflection is specular; a ray reflects at most R_max times
// (Tables 2 and 3) and ends when its arc length reaches s_max.
//
// Every floating-point step is a single IEEE double operation in a fixed
// order (no contraction into fused multiply-adds): the table is the same,
// bit for bit, whatever the launch shape, and a reference that performs the
// same operations reproduces it exactly.
//
// Box search: boxes are grouped (host side) into spatially compact groups
// of kTraceGroup with a bounding box each.  A group's slab interval contains
// the interval of every member (rounding is monotone), so the group test
// never rejects a member that would be hit.  Groups and members are read
// with wave-uniform indices.
//
// Two launches of the same kernel: the count pass writes each ray's segment
// count; after a prefix sum the write pass traces again and stores the
// segments at the ray's offset.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gbs_internal.h"

#pragma clang fp contract(off)

namespace gbs {

namespace {

constexpr double kTraceEps = 1e-7;          // minimum hit distance (no self-hits)

struct Slab {
    double tnear, tfar;
    double tmin0, tmin1, tmin2;
};

// Interval of t where p + t d lies inside [lo, hi] (per axis, then
// intersected), with the per-axis entries for the entry-axis rule.
__device__ __forceinline__ Slab slab(const double p[3], const double d[3], const double inv[3], const double lo[3],
                                     const double hi[3]) {
    double tmin[3], tmax[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (d[j] == 0.0) {
            const bool inside = lo[j] <= p[j] && p[j] <= hi[j];
            tmin[j] = inside ? -INFINITY : INFINITY;
            tmax[j] = inside ? INFINITY : -INFINITY;
        } else {
            const double t1 = (lo[j] - p[j]) * inv[j];
            const double t2 = (hi[j] - p[j]) * inv[j];
            tmin[j] = t1 < t2 ? t1 : t2;
            tmax[j] = t1 > t2 ? t1 : t2;
        }
    }
    // max(max(a, b), c) and min(min(a, b), c), first argument kept on ties
    double tn = tmin[1] > tmin[0] ? tmin[1] : tmin[0];
    tn = tmin[2] > tn ? tmin[2] : tn;
    double tf = tmax[1] < tmax[0] ? tmax[1] : tmax[0];
    tf = tmax[2] < tf ? tmax[2] : tf;
    return Slab{tn, tf, tmin[0], tmin[1], tmin[2]};
}

__device__ __forceinline__ int32_t face_of(int32_t box, const double* bx, int axis, int side, const double hp[3],
                                           int panels) {
    const int wall = axis == 0 ? (side == 0 ? 0 : 1) : axis == 1 ? (side == 0 ? 2 : 3) : 4;
    int cell = 0;
    if (panels > 1) {
        const double x0 = bx[0], x1 = bx[1], y0 = bx[2], y1 = bx[3], h = bx[4];
        const double u = axis == 0 ? (hp[1] - y0) / (y1 - y0) : (hp[0] - x0) / (x1 - x0);
        const double v = axis == 2 ? (hp[1] - y0) / (y1 - y0) : hp[2] / h;
        int iu = (int)(u * (double)panels), iv = (int)(v * (double)panels);
        iu = iu < 0 ? 0 : (iu > panels - 1 ? panels - 1 : iu);
        iv = iv < 0 ? 0 : (iv > panels - 1 ? panels - 1 : iv);
        cell = iu * panels + iv;
    }
    return 1 + box * 5 * panels * panels + wall * panels * panels + cell;
}

}  // namespace

// One thread per ray.  COUNT: nseg[i] = segments of ray i; bad[0] gets bit 0
// for a direction that is not a unit vector, bit 1 for a source index out of
// range or out of order (the index is clamped for the reads meanwhile), bit 2
// for a launch frame (e1_in) that is not a unit vector normal to the
// direction.  Otherwise the segments are
// written from ray_ptr[i]; their face histories from face_base[i] (segment j
// of a ray holds j faces, at face_base + j (j - 1) / 2).
//   boxes   [n_boxes * 5] x0, x1, y0, y1, h in the caller's order
//   gbox    [n_groups * 6] group bounds lo xyz, hi xyz
//   members [n_groups * kTraceGroup] box index per group slot (-1 = empty)
template <bool COUNT>
__global__ __launch_bounds__(kTraceThreads) void k_trace(
    int64_t n_rays, int n_src, const double* __restrict__ src_xyz, const int32_t* __restrict__ ray_src,
    const double* __restrict__ dirs, const double* __restrict__ s_max_src, const double* __restrict__ boxes,
    const double* __restrict__ gbox, const int32_t* __restrict__ members, int n_groups, int panels, int max_refl,
    double s_max_all, int image_complete,
    int64_t* __restrict__ nseg, int* __restrict__ bad, const int64_t* __restrict__ ray_ptr,
    const int64_t* __restrict__ face_base, double* __restrict__ seg_a, double* __restrict__ seg_t,
    double* __restrict__ seg_s0, double* __restrict__ seg_lo, double* __restrict__ seg_hi,
    int64_t* __restrict__ face_ptr, int32_t* __restrict__ face_ids, const double* __restrict__ e1_in,
    double* __restrict__ seg_e1) {
    __shared__ int32_t hist_s[kTraceMaxRefl * kTraceThreads];   // face history: slot j * threads + tid
    const int64_t i = (int64_t)blockIdx.x * kTraceThreads + threadIdx.x;
    const bool live = i < n_rays;
    const int64_t ii = live ? i : 0;
    const int sraw = ray_src ? ray_src[ii] : 0;
    const int sidx = sraw < 0 ? 0 : (sraw >= n_src ? n_src - 1 : sraw);
    const double src[3] = {src_xyz[3 * sidx], src_xyz[3 * sidx + 1], src_xyz[3 * sidx + 2]};
    const double d0[3] = {dirs[3 * ii], dirs[3 * ii + 1], dirs[3 * ii + 2]};
    const double s_max = s_max_src ? s_max_src[sidx] : s_max_all;    // the ray's arc-length budget
    if (COUNT && live) {
        const double n2 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2];
        int flag = fabs(n2 - 1.0) <= 1e-9 ? 0 : 1;
        if (sraw != sidx || (ray_src && ii > 0 && ray_src[ii - 1] > sraw)) flag |= 2;
        if (e1_in) {
            const double en = e1_in[3 * ii] * e1_in[3 * ii] + e1_in[3 * ii + 1] * e1_in[3 * ii + 1] +
                              e1_in[3 * ii + 2] * e1_in[3 * ii + 2];
            const double ed = e1_in[3 * ii] * d0[0] + e1_in[3 * ii + 1] * d0[1] + e1_in[3 * ii + 2] * d0[2];
            if (!(fabs(en - 1.0) <= 1e-9 && fabs(ed) <= 1e-9)) flag |= 4;
        }
        if (flag) atomicOr(bad, flag);
    }
    double p[3] = {src[0], src[1], src[2]};
    double d[3] = {d0[0], d0[1], d0[2]};
    // launch frame (anisotropic beams), mirrored at every reflection like d
    const double e0[3] = {e1_in ? e1_in[3 * ii] : 0.0, e1_in ? e1_in[3 * ii + 1] : 0.0,
                          e1_in ? e1_in[3 * ii + 2] : 0.0};
    double e[3] = {e0[0], e0[1], e0[2]};
    double s = 0.0;
    int n = 0;
    bool any_ground = false;
    // the previous segment, written once the next one is known (its hi
    // extends through a ground reflection)
    double pa[3] = {0, 0, 0}, pt[3] = {0, 0, 0}, pe[3] = {0, 0, 0}, ps0 = 0.0, plo = 0.0, pL = 0.0;
    bool pground = false;
    const int64_t out0 = (!COUNT && live) ? ray_ptr[ii] : 0;
    const int64_t f0 = (!COUNT && live) ? face_base[ii] : 0;
    auto emit = [&](int j, const double a[3], const double t[3], const double fe[3], double s0, double lo,
                    double hi) {
        const int64_t o = out0 + j;
        if (seg_e1) {
            seg_e1[3 * o] = fe[0];
            seg_e1[3 * o + 1] = fe[1];
            seg_e1[3 * o + 2] = fe[2];
        }
        seg_a[3 * o] = a[0];
        seg_a[3 * o + 1] = a[1];
        seg_a[3 * o + 2] = a[2];
        seg_t[3 * o] = t[0];
        seg_t[3 * o + 1] = t[1];
        seg_t[3 * o + 2] = t[2];
        seg_s0[o] = s0;
        seg_lo[o] = lo;
        seg_hi[o] = hi;
        const int64_t fo = f0 + (int64_t)j * (j - 1) / 2;
        face_ptr[o] = fo;
        for (int m = 0; m < j; ++m) face_ids[fo + m] = hist_s[m * kTraceThreads + threadIdx.x];
    };
    bool done = !live;
    for (int k = 0; k <= max_refl; ++k) {
        // every thread takes part in the wave-uniform group loop; finished rays
        // just ignore the results
        double inv[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) inv[j] = d[j] != 0.0 ? 1.0 / d[j] : 0.0;
        double tg = d[2] < 0.0 ? -p[2] / d[2] : INFINITY;
        if (!(tg > kTraceEps)) tg = INFINITY;
        double best = tg;
        int32_t best_box = -1;
        int best_axis = 0, best_side = 0;
        if (k < max_refl && __any(!done)) {
            for (int g = 0; g < n_groups; ++g) {
                const double* gb = gbox + 6 * g;
                const double glo[3] = {gb[0], gb[1], gb[2]}, ghi[3] = {gb[3], gb[4], gb[5]};
                const Slab G = slab(p, d, inv, glo, ghi);
                if (!(G.tnear <= G.tfar && G.tfar > kTraceEps && G.tnear <= best) || done) continue;
                for (int m = 0; m < kTraceGroup; ++m) {
                    const int32_t b = members[g * kTraceGroup + m];
                    if (b < 0) break;
                    const double* bx = boxes + 5 * (int64_t)b;
                    const double lo[3] = {bx[0], bx[2], 0.0}, hi[3] = {bx[1], bx[3], bx[4]};
                    const Slab S = slab(p, d, inv, lo, hi);
                    if (!(S.tnear <= S.tfar && S.tnear > kTraceEps)) continue;
                    const int axis = (S.tmin0 >= S.tmin1 && S.tmin0 >= S.tmin2) ? 0 : (S.tmin1 >= S.tmin2 ? 1 : 2);
                    if (axis == 2 && d[2] > 0.0) continue;          // through the floor
                    // nearest; the ground (best_box < 0) and lower box indices win ties
                    if (S.tnear < best || (S.tnear == best && best_box >= 0 && b < best_box)) {
                        best = S.tnear;
                        best_box = b;
                        best_axis = axis;
                        best_side = d[axis] > 0.0 ? 0 : 1;
                    }
                }
            }
        }
        if (done) continue;
        const double remaining = s_max - s;
        const bool ends = best >= remaining || k == max_refl;
        const double L = ends ? remaining : best;
        double hp[3] = {p[0] + L * d[0], p[1] + L * d[1], p[2] + L * d[2]};
        const bool ground = !ends && best_box < 0;
        int32_t face = -1;
        if (!ends) face = ground ? 0 : face_of(best_box, boxes + 5 * (int64_t)best_box, best_axis, best_side, hp,
                                               panels);
        if (!COUNT) {
            if (n > 0) emit(n - 1, pa, pt, pe, ps0, plo, pground ? pL + L : pL);
            pa[0] = p[0]; pa[1] = p[1]; pa[2] = p[2];
            pt[0] = d[0]; pt[1] = d[1]; pt[2] = d[2];
            pe[0] = e[0]; pe[1] = e[1]; pe[2] = e[2];
            ps0 = s;
            plo = (n > 0 && pground) ? -pL : 0.0;
            pL = L;
            pground = ground;
            if (!ends) hist_s[n * kTraceThreads + threadIdx.x] = face;
        }
        ++n;
        any_ground |= ground;
        if (ends) {
            done = true;
            continue;
        }
        const int ax = ground ? 2 : best_axis;
        d[ax] = -d[ax];
        e[ax] = -e[ax];
        if (ground) hp[2] = 0.0;
        p[0] = hp[0]; p[1] = hp[1]; p[2] = hp[2];
        s = s + L;
    }
    if (!live) return;
    const bool image = image_complete && !any_ground;
    if (COUNT) {
        nseg[i] = n + (image ? 1 : 0);
        return;
    }
    emit(n - 1, pa, pt, pe, ps0, plo, pL);
    if (image) {
        if (seg_e1) {
            const int64_t oi = out0 + n;
            seg_e1[3 * oi] = e0[0];
            seg_e1[3 * oi + 1] = e0[1];
            seg_e1[3 * oi + 2] = -e0[2];
        }
        const double a[3] = {src[0], src[1], -src[2]};
        const double t[3] = {d0[0], d0[1], -d0[2]};
        const int64_t o = out0 + n;
        seg_a[3 * o] = a[0];
        seg_a[3 * o + 1] = a[1];
        seg_a[3 * o + 2] = a[2];
        seg_t[3 * o] = t[0];
        seg_t[3 * o + 1] = t[1];
        seg_t[3 * o + 2] = t[2];
        seg_s0[o] = 0.0;
        seg_lo[o] = 0.0;
        seg_hi[o] = s_max;
        const int64_t fo = f0 + (int64_t)n * (n - 1) / 2;
        face_ptr[o] = fo;
        face_ids[fo] = 0;
    }
}

// Face-history length of every ray: sum over its segments j of j.
__global__ void k_trace_face_counts(int64_t n_rays, const int64_t* __restrict__ nseg, int64_t* __restrict__ nface) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > n_rays) return;
    const int64_t n = i < n_rays ? nseg[i] : 0;
    nface[i] = n * (n - 1) / 2;
}

// The closing entry of face_ptr.
__global__ void k_trace_close(const int64_t* __restrict__ face_base, int64_t n_rays, int64_t n_segs,
                              int64_t* __restrict__ face_ptr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) face_ptr[n_segs] = face_base[n_rays];
}

template __global__ void k_trace<true>(int64_t, int, const double*, const int32_t*, const double*, const double*,
                                       const double*,
                                       const double*, const int32_t*, int, int, int, double, int, int64_t*, int*,
                                       const int64_t*, const int64_t*, double*, double*, double*, double*, double*,
                                       int64_t*, int32_t*, const double*, double*);
template __global__ void k_trace<false>(int64_t, int, const double*, const int32_t*, const double*, const double*,
                                        const double*,
                                        const double*, const int32_t*, int, int, int, double, int, int64_t*, int*,
                                        const int64_t*, const int64_t*, double*, double*, double*, double*, double*,
                                        int64_t*, int32_t*, const double*, double*);

}  // namespace gbs

// gfx950 kernels of libgbs: receiver ordering, segment preparation, culled
// work lists and the persistent beam-summation kernels (forward and adjoint).
//
// Work decomposition.  The paper balances its ragged per-observer beam loops
// with device-side kernel launches (Sec. 3.4).  Here the ragged work becomes
// explicit lists: receivers are ordered along a Morton curve and cut into
// patches; for every (job, patch) a culling pass lists the segments whose
// Gaussian beam can reach any receiver of the patch; an exclusive prefix sum
// over the list lengths lays the lists out back to back; a persistent kernel
// drains (job, patch) items, longest first, with an atomic counter.
//
// Pair kernel layout.  One wavefront per item, one receiver per lane (or
// several, NR).  The item's segment list is wave-uniform, so segment records
// stream through scalar loads into SGPRs and every lane reads them without
// LDS traffic; each lane keeps its receivers and FP64 running sums in VGPRs.
#include "gbs_internal.h"

#include <math.h>

#include <type_traits>

namespace gbs {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double wave_min(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
// Wave sums with data-parallel-primitive lane moves (no LDS traffic): an
// inclusive scan inside each row of 16 lanes (row_shr 1, 2, 4, 8), then the
// row totals carried by row_bcast 15 and 31.  The full sum ends up in the
// last lane only; other lanes hold partial sums.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(dpp_i32<CTRL, ROWS>(__float_as_int(v)));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL, ROWS>((int)(u & 0xffffffffll)), hi = dpp_i32<CTRL, ROWS>((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T>
__device__ __forceinline__ T wave_sum_last(T v) {
    constexpr bool kD = sizeof(T) == 8;
    if constexpr (kD) {
        v += dpp_f64<0x111, 0xf>(v);
        v += dpp_f64<0x112, 0xf>(v);
        v += dpp_f64<0x114, 0xf>(v);
        v += dpp_f64<0x118, 0xf>(v);
        v += dpp_f64<0x142, 0xa>(v);
        v += dpp_f64<0x143, 0xc>(v);
    } else {
        v += dpp_f32<0x111, 0xf>(v);
        v += dpp_f32<0x112, 0xf>(v);
        v += dpp_f32<0x114, 0xf>(v);
        v += dpp_f32<0x118, 0xf>(v);
        v += dpp_f32<0x142, 0xa>(v);
        v += dpp_f32<0x143, 0xc>(v);
    }
    return v;
}

// The sum over each row of 16 lanes, left in the row's last lane.
template <typename T>
__device__ __forceinline__ T row_sum_last(T v) {
    if constexpr (sizeof(T) == 8) {
        v += dpp_f64<0x111, 0xf>(v);
        v += dpp_f64<0x112, 0xf>(v);
        v += dpp_f64<0x114, 0xf>(v);
        v += dpp_f64<0x118, 0xf>(v);
    } else {
        v += dpp_f32<0x111, 0xf>(v);
        v += dpp_f32<0x112, 0xf>(v);
        v += dpp_f32<0x114, 0xf>(v);
        v += dpp_f32<0x118, 0xf>(v);
    }
    return v;
}

// An empty volatile asm has side effects, so the compiler cannot hoist the
// gated block above its wave-uniform branch and execute it for every pair.
__device__ __forceinline__ void branch_barrier() { asm volatile(""); }

// Orders this wave's LDS accesses around a tile hand-over: the tile slice is
// private to the wave and LDS executes one wave's operations in order, so a
// compiler-level fence is all that is needed.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// An empty asm that takes v and hands it back in the same registers: the
// compiler waits for v's load before it, and afterwards v is no longer a load
// in flight, so a loop that reads it has no wait of its own (a value loaded
// before a loop is otherwise waited for at each store in it, and on gfx9 the
// wait covers the earlier stores as well).  The memory clobber keeps the
// stores issued before it in front of it.
template <typename T>
__device__ __forceinline__ void settle(T& v) { asm volatile("" : "+v"(v) : : "memory"); }

__device__ __forceinline__ int lanes_before(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Exact accumulation (see Fixed): adds x scaled by `scale` = 2^K.  The split
// y = hi 2^32 + lo is exact: fma forms y - hi 2^32 with one rounding, and that
// difference is representable.
__device__ __forceinline__ void fixed_add(Fixed* acc, double x, double scale) {
    const double y = x * scale;
    const double h = floor(y * 0x1p-32);
    const double l = fma(-h, 0x1p32, y);
    atomicAdd(&acc->hi, (unsigned long long)(long long)h);
    atomicAdd(&acc->lo, (unsigned long long)(long long)l);
}
// The accumulated value times inv_scale = 2^-K (deterministic rounding).
__device__ __forceinline__ double fixed_value(const Fixed& acc, double inv_scale) {
    const long long l = (long long)acc.lo;
    const long long h = (long long)acc.hi + (l >> 32);
    return fma((double)h, 0x1p32, (double)(l & 0xffffffffll)) * inv_scale;
}
// 2^K with K the largest integer such that bound * 2^K <= 2^kFixedBits
// (bound <= 0 or not finite: 1).
__device__ __forceinline__ double fixed_scale_for(double bound) {
    if (!(bound > 0.0) || !isfinite(bound)) return 1.0;
    return ldexp(1.0, kFixedBits - 1 - ilogb(bound));
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_reset_counter(unsigned* ctr) { *ctr = 0u; }

// ---------------------------------------------------------------- receivers
// Bounding box of the receivers: per-block partial min/max, then one block.
__global__ void k_bbox_partial(const double* __restrict__ rcv, int64_t n, double* __restrict__ part) {
    __shared__ double sm[6][256];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            double x = rcv[3 * i + d];
            lo[d] = fmin(lo[d], x);
            hi[d] = fmax(hi[d], x);
        }
    }
    for (int d = 0; d < 3; ++d) {
        sm[d][threadIdx.x] = lo[d];
        sm[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                sm[d][threadIdx.x] = fmin(sm[d][threadIdx.x], sm[d][threadIdx.x + s]);
                sm[3 + d][threadIdx.x] = fmax(sm[3 + d][threadIdx.x], sm[3 + d][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) part[6 * blockIdx.x + d] = sm[d][0];
}

__global__ __launch_bounds__(256) void k_bbox_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ bbox) {
    __shared__ double sm[6][256];
    double b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        for (int d = 0; d < 3; ++d) {
            b[d] = fmin(b[d], part[6 * i + d]);
            b[3 + d] = fmax(b[3 + d], part[6 * i + 3 + d]);
        }
    for (int d = 0; d < 6; ++d) sm[d][threadIdx.x] = b[d];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                sm[d][threadIdx.x] = fmin(sm[d][threadIdx.x], sm[d][threadIdx.x + s]);
                sm[3 + d][threadIdx.x] = fmax(sm[3 + d][threadIdx.x], sm[3 + d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) bbox[d] = sm[d][0];
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ void k_morton(const double* __restrict__ rcv, int64_t n, const double* __restrict__ bbox,
                         uint32_t* __restrict__ keys, int32_t* __restrict__ vals) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double ext = bbox[3 + d] - bbox[d];
        double u = ext > 0 ? (rcv[3 * i + d] - bbox[d]) / ext : 0.0;
        q[d] = (uint32_t)fmin(fmax(u * 1023.0, 0.0), 1023.0);
    }
    keys[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
    vals[i] = (int32_t)i;
}

// Sorted receivers in SoA, padded to whole patches with copies of the last
// receiver (perm = -1 marks padding, whose results are discarded).
__global__ void k_gather_rcv(const double* __restrict__ rcv, int64_t n, int64_t n_pad,
                             const int32_t* __restrict__ order, double* __restrict__ rx, double* __restrict__ ry,
                             double* __restrict__ rz, double* __restrict__ r2, int32_t* __restrict__ perm,
                             int* __restrict__ status) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    int32_t o = order[i < n ? i : n - 1];
    double x = rcv[3 * (int64_t)o], y = rcv[3 * (int64_t)o + 1], z = rcv[3 * (int64_t)o + 2];
    if (i < n && !(isfinite(x) && isfinite(y) && isfinite(z))) atomicOr(status, kBadReceiver);
    rx[i] = x;
    ry[i] = y;
    rz[i] = z;
    r2[i] = x * x + y * y + z * z;
    perm[i] = i < n ? o : -1;
}

// Bounding sphere of each group of `per` consecutive sorted receivers; one
// wavefront per group.
__global__ __launch_bounds__(64) void k_patches(const double* __restrict__ rx, const double* __restrict__ ry,
                                                const double* __restrict__ rz, int64_t n_pad, int64_t per,
                                                int n_groups, Patch* __restrict__ out) {
    const int g = blockIdx.x;
    if (g >= n_groups) return;
    const int lane = threadIdx.x;
    const int64_t b = (int64_t)g * per, e = b + per < n_pad ? b + per : n_pad;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = b + lane; i < e; i += 64) {
        double v[3] = {rx[i], ry[i], rz[i]};
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], v[d]);
            hi[d] = fmax(hi[d], v[d]);
        }
    }
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = 0.5 * (wave_min(lo[d]) + wave_max(hi[d]));
    double r = 0.0;
    for (int64_t i = b + lane; i < e; i += 64) {
        double dx = rx[i] - c[0], dy = ry[i] - c[1], dz = rz[i] - c[2];
        r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
    }
    r = wave_max(r);
    if (lane == 0) out[g] = Patch{c[0], c[1], c[2], r};
}

// Bounding sphere of each group of `per` consecutive child spheres (one
// wavefront per group): centre at the middle of the children's box, radius
// the farthest child surface point, so it holds every child's receivers.
__global__ __launch_bounds__(64) void k_sphere_of_spheres(const Patch* __restrict__ child, int n_child, int per,
                                                          int n_groups, Patch* __restrict__ out) {
    const int g = blockIdx.x;
    if (g >= n_groups) return;
    const int lane = threadIdx.x;
    const int b = g * per, e = min(b + per, n_child);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = b + lane; i < e; i += 64) {
        const Patch c = child[i];
        const double v[3] = {c.cx, c.cy, c.cz};
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], v[d] - c.rad);
            hi[d] = fmax(hi[d], v[d] + c.rad);
        }
    }
    double C[3];
    for (int d = 0; d < 3; ++d) C[d] = 0.5 * (wave_min(lo[d]) + wave_max(hi[d]));
    double r = 0.0;
    for (int i = b + lane; i < e; i += 64) {
        const Patch c = child[i];
        const double dx = c.cx - C[0], dy = c.cy - C[1], dz = c.cz - C[2];
        r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz) + c.rad);
    }
    r = wave_max(r);
    if (lane == 0) out[g] = Patch{C[0], C[1], C[2], r * (1.0 + 1e-12)};
}

// ----------------------------------------------------------------- segments
// First segment of every source (rays are sorted by source); src_off[n_src]
// is the end of the table.
// Also checks the ray CSR (ray_ptr[0] = 0, non-decreasing, ray_ptr[n_rays] =
// n_segs), the source order and face_ptr[0] = 0.
__global__ void k_src_ranges(const int64_t* __restrict__ ray_ptr, const int32_t* __restrict__ ray_src,
                             int64_t n_rays, int32_t n_src, int64_t n_segs, const int64_t* __restrict__ face_ptr,
                             int face_ids_given, int32_t n_faces, int64_t* __restrict__ src_off,
                             int* __restrict__ status) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > n_rays) return;
    const int32_t rp = i == 0 ? -1 : ray_src[i - 1], rc = i == n_rays ? n_src : ray_src[i];
    int bad = 0;
    if ((i > 0 && (rp < 0 || rp >= n_src)) || rc < rp) bad |= kBadRaySource;
    const int64_t p = ray_ptr[i];
    if (i == 0 ? p != 0 : p < ray_ptr[i - 1]) bad |= kBadRayPtr;
    if (i == n_rays && p != n_segs) bad |= kBadRayPtr;
    if (i == 0 && face_ptr) {
        const int64_t total = face_ptr[n_segs];
        if (face_ptr[0] != 0 || total < 0 || (total > 0 && !face_ids_given)) bad |= kBadFacePtr;
        if (total > 0 && n_faces <= 0) bad |= kBadFaceId;
    }
    if (bad) atomicOr(status, bad);
    // clamped so that an unsorted or out-of-range table cannot write outside src_off
    int32_t prev = min(max(rp, -1), n_src);
    int32_t cur = min(max(rc, -1), n_src);
    for (int32_t s = prev + 1; s <= cur; ++s) src_off[s] = p;
}

// Per-job constants of one pass (one thread per job), from the band
// frequencies, the beam parameters, the optional absorption and second beam
// parameter, and the sources' segment ranges; flags invalid job inputs.
// Anisotropic beams: the cull and the pre-gate use the envelope of the two
// widths (it keeps every pair the exact gate keeps), widened by a relative
// 1e-12 against rounding; the pair kernel applies the exact gate.
__global__ void k_job_consts(const double* __restrict__ freqs, const double* __restrict__ eps,
                             const double* __restrict__ alpha, const double* __restrict__ eps_e2, int32_t n_src,
                             int32_t n_freq, double c, double G, const int64_t* __restrict__ src_off,
                             int64_t pass_begin, int64_t pass_end, JobConst* __restrict__ jobs,
                             int* __restrict__ status) {
    const int job = blockIdx.x * blockDim.x + threadIdx.x;
    if (job >= n_src * n_freq) return;
    const int s = job / n_freq, b = job - s * n_freq;
    constexpr double pi = 3.14159265358979323846, log2e = 1.4426950408889634;
    const double f = freqs[b], e = eps[job], al = alpha ? alpha[job] : 0.0, eb = eps_e2 ? eps_e2[job] : e;
    if (!(isfinite(f) && f > 0.0 && isfinite(e) && e > 0.0 && isfinite(al) && al >= 0.0 && isfinite(eb) &&
          eb > 0.0))
        atomicOr(status, kBadJob);
    const double k = 2.0 * pi * f / c;
    const double ke = k * e;
    JobConst j;
    j.seg_begin = max(src_off[s], pass_begin) - pass_begin;
    j.seg_end = min(src_off[s + 1], pass_end) - pass_begin;
    if (j.seg_end < j.seg_begin) j.seg_end = j.seg_begin;
    j.k = k;
    j.eps = e;
    j.eps2 = e * e;
    j.gate_c1 = 1.0 + 2.0 * G / ke;
    j.gate_c2 = 2.0 * G * e * e / ke;
    j.kappa = 2.0 * G / ke;
    j.fk = f / c;
    j.hfk = 0.5 * f / c;
    j.gexp2 = -0.5 * ke * log2e;
    j.gexp = -0.5 * ke;
    j.scale = ke / (8.0 * pi * pi);
    j.aexp = -al;
    j.aexp2 = j.aexp * log2e;
    j.epsb = e;
    j.epsa2 = e * e;
    j.epsb2 = e * e;
    j.gate_a = 2.0 * G / k;
    j.gexpa = -0.5 * k;
    j.gexpa2 = -0.5 * k * log2e;
    j.ampc = 0.5 * e;
    if (eps_e2) {
        const double margin = 1.0 + 1e-12;
        j.epsb = eb;
        j.epsb2 = eb * eb;
        j.ampc = 0.5 * sqrt(e * eb);
        j.kappa = 2.0 * G / (k * fmin(e, eb)) * margin;
        j.eps2 = e * eb * margin;
        j.gate_c1 = 1.0 + j.kappa;
        j.gate_c2 = j.kappa * j.eps2;
        j.scale = k / (8.0 * pi * pi);
    }
    j.src = s;
    j.band = b;
    jobs[job] = j;
}

// The cull's pieces of a pass: every source's segment range [src_off[s],
// src_off[s+1]) inside the pass cut into pieces of `span` segments, in source
// order (one thread; at most n_src + n_segs / span pieces).
__global__ void k_make_splits(const int64_t* __restrict__ src_off, int32_t n_src, int64_t pass_begin,
                              int64_t pass_end, int64_t span, int32_t max_splits, int64_t cells,
                              CullSplit* __restrict__ splits, int32_t* __restrict__ n_splits,
                              int64_t* __restrict__ src_cnt) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int32_t n = 0;
    for (int32_t s = 0; s < n_src; ++s) {
        const int64_t b = max(src_off[s], pass_begin) - pass_begin, e = min(src_off[s + 1], pass_end) - pass_begin;
        int32_t k = 0;
        src_cnt[2 * s] = (int64_t)n * cells;
        for (int64_t x = b; x < e && n < max_splits; x += span, ++k)
            splits[n++] = CullSplit{x, min(x + span, e), s, k};
        src_cnt[2 * s + 1] = k;
    }
    *n_splits = n;
}

// seg_ray[j] = index (within the pass) of the ray that owns segment j.
__global__ void k_seg2ray(const int64_t* __restrict__ ray_ptr, int64_t n_rays, int64_t seg_base, int64_t n_segs,
                          int32_t* __restrict__ seg_ray) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n_rays) return;
    const int64_t b = max(ray_ptr[i] - seg_base, (int64_t)0), e = min(ray_ptr[i + 1] - seg_base, n_segs);
    for (int64_t j = b; j < e; ++j) seg_ray[j] = (int32_t)i;
}

// Segment records: virtual-source anchoring, arc-length interval and the
// complex weight w * prod(Gamma) over the faces hit before the segment.
// Checks the segment's values, its face-history range (inside
// [face_base, face_end], absolute offsets; face_end read from face_end_p when
// given) and ids, and its ray (status bits); bad
// entries are skipped, never read out of range.  With bmax, also the largest
// w * (history length) * prod max(1, |Gamma|) over the pass (a bound on the
// coefficient derivatives, for the adjoint's exact face sums).
__global__ void k_records(int64_t n_segs, const double* __restrict__ a, const double* __restrict__ t,
                          const double* __restrict__ s0, const double* __restrict__ lo,
                          const double* __restrict__ hi, const int64_t* __restrict__ face_ptr,
                          int64_t face_base, const int32_t* __restrict__ face_ids, int32_t n_faces,
                          const double* __restrict__ gamma, const double* __restrict__ ray_w,
                          const int32_t* __restrict__ seg_ray, int64_t n_rays,
                          const int64_t* __restrict__ face_end_p, int64_t face_end_h, SegRec* __restrict__ rec,
                          int* __restrict__ status, unsigned long long* __restrict__ bmax) {
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_segs) return;
    int bad = 0;
    double tx = t[3 * j], ty = t[3 * j + 1], tz = t[3 * j + 2];
    double s = s0[j];
    const double ax = a[3 * j], ay = a[3 * j + 1], az = a[3 * j + 2], l0 = lo[j], l1 = hi[j];
    const double tn = tx * tx + ty * ty + tz * tz;
    if (!(isfinite(ax) && isfinite(ay) && isfinite(az) && isfinite(s) && isfinite(l0) && isfinite(l1) &&
          l0 <= l1 && fabs(tn - 1.0) <= 2e-9))
        bad |= kBadSegment;
    double ox = ax - s * tx, oy = ay - s * ty, oz = az - s * tz;
    const int32_t ray = seg_ray[j];
    double gr = 0.0, gi = 0.0;
    if (ray < 0 || ray >= n_rays) {
        bad |= kBadRayPtr;
    } else {
        gr = ray_w[ray];
        if (!(isfinite(gr) && gr >= 0.0)) bad |= kBadRayWeight;
    }
    const int64_t f0 = face_ptr[j], f1 = face_ptr[j + 1];
    const int64_t face_end = face_end_p ? *face_end_p : face_end_h;
    double gmax = 1.0;
    if (!(face_base <= f0 && f0 <= f1 && f1 <= face_end)) {
        bad |= kBadFacePtr;
    } else {
        for (int64_t m = f0 - face_base; m < f1 - face_base; ++m) {
            const int32_t f = face_ids[m];
            if (f < 0 || f >= n_faces) {
                bad |= kBadFaceId;
                continue;
            }
            double xr = gamma[2 * f], xi = gamma[2 * f + 1];
            double nr = gr * xr - gi * xi;
            gi = gr * xi + gi * xr;
            gr = nr;
            gmax *= fmax(1.0, hypot(xr, xi));
        }
    }
    if (bad) atomicOr(status, bad);
    if (bmax) {
        const double b = (ray >= 0 && ray < n_rays ? fabs(ray_w[ray]) : 0.0) * (double)(f1 - f0) * gmax;
        if (b > 0.0 && isfinite(b)) atomicMax(bmax, (unsigned long long)__double_as_longlong(b));
    }
    SegRec r;
    r.m2ox = -2.0 * ox;
    r.m2oy = -2.0 * oy;
    r.m2oz = -2.0 * oz;
    r.oo = ox * ox + oy * oy + oz * oz;
    r.tx = tx;
    r.ty = ty;
    r.tz = tz;
    r.mot = -(ox * tx + oy * ty + oz * tz);
    r.slo = s + l0;
    r.shi = s + l1;
    r.wgr = gr;
    r.wgi = gi;
    r.wph = atan2(gi, gr) * (0.5 / 3.14159265358979323846);
    r.pad = 0.0;
    rec[j] = r;
}

// Spatial order of the segments of a pass: key = (source << 32) | 30-bit
// Morton code of the beam interval's midpoint, clamped to the receivers'
// bounding box.  Chunks of consecutive segments then reach few hyper-patches
// together, which lets the cull skip them.  The source of segment j is found
// from the per-job segment ranges (jobs[s * n_freq] for source s).
__global__ void k_seg_keys(int64_t n_segs, const SegRec* __restrict__ rec, const JobConst* __restrict__ jobs,
                           int32_t n_src, int32_t n_freq, const double* __restrict__ bbox,
                           unsigned long long* __restrict__ keys, int32_t* __restrict__ ids) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_segs) return;
    const SegRec S = rec[j];
    const double h = 0.5 * (S.slo + S.shi);
    const double m[3] = {-0.5 * S.m2ox + h * S.tx, -0.5 * S.m2oy + h * S.ty, -0.5 * S.m2oz + h * S.tz};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        const double ext = bbox[3 + d] - bbox[d];
        const double u = ext > 0 ? (m[d] - bbox[d]) / ext : 0.0;
        q[d] = (uint32_t)fmin(fmax(u * 1023.0, 0.0), 1023.0);
    }
    int32_t src = 0;
    for (int s = 0; s < n_src; ++s)
        if (j >= jobs[(int64_t)s * n_freq].seg_begin) src = s;
    keys[j] = ((unsigned long long)src << 32) | (spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2));
    ids[j] = (int32_t)j;
}

// out[i] = in[perm[i]] for 96-byte segment records.
__global__ void k_permute_rec(int64_t n, const SegRec* __restrict__ in, const int32_t* __restrict__ perm,
                              SegRec* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = in[perm[i]];
}

// Ray frames of a pass (table order): e1 given per segment (checked: unit and
// normal to t within 1e-9), or, without one, e1 = z x t / |z x t| (the x axis
// when t is vertical); e2 = t x e1; -o.e_m with o = a - s0 t.
__global__ void k_frames(int64_t n_segs, const double* __restrict__ a, const double* __restrict__ t,
                         const double* __restrict__ s0, const double* __restrict__ e1, FrameRec* __restrict__ out,
                         int* __restrict__ status) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n_segs) return;
    const double tx = t[3 * j], ty = t[3 * j + 1], tz = t[3 * j + 2];
    double ex, ey, ez;
    if (e1) {
        ex = e1[3 * j];
        ey = e1[3 * j + 1];
        ez = e1[3 * j + 2];
        const double nn = ex * ex + ey * ey + ez * ez, d = ex * tx + ey * ty + ez * tz;
        if (!(fabs(nn - 1.0) <= 2e-9 && fabs(d) <= 1e-9)) atomicOr(status, kBadSegment);
    } else {
        const double h2 = fma(tx, tx, ty * ty);
        ex = 1.0;
        ey = 0.0;
        ez = 0.0;
        if (h2 > 0.0) {
            const double rh = 1.0 / sqrt(h2);
            ex = -ty * rh;
            ey = tx * rh;
        }
    }
    const double fx = ty * ez - tz * ey, fy = tz * ex - tx * ez, fz = tx * ey - ty * ex;
    const double s = s0[j];
    const double ox = a[3 * j] - s * tx, oy = a[3 * j + 1] - s * ty, oz = a[3 * j + 2] - s * tz;
    FrameRec f;
    f.e1x = ex;
    f.e1y = ey;
    f.e1z = ez;
    f.moe1 = -(ox * ex + oy * ey + oz * ez);
    f.e2x = fx;
    f.e2y = fy;
    f.e2z = fz;
    f.moe2 = -(ox * fx + oy * fy + oz * fz);
    out[j] = f;
}

// out[i] = in[perm[i]] for frame records.
__global__ void k_permute_frames(int64_t n, const FrameRec* __restrict__ in, const int32_t* __restrict__ perm,
                                 FrameRec* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = in[perm[i]];
}

// ------------------------------------------------------------------ culling
// Conservative test: can the beam of segment S pass the gate for any receiver
// inside a bounding sphere (centre C, radius rad)?  For R in the sphere, the
// arc length is within rad of the centre's and the normal distance is at
// least the centre's minus rad (distance to a line is 1-Lipschitz), while
// the gate needs n^2 <= kappa (s^2 + eps^2).  The geometry does not depend on
// the band; each band then only compares d^2 <= kappa_b sm^2 + kappa_b eps_b^2
// with d = max(n_C - rad, 0) and sm the largest |s| the sphere can reach
// inside the beam interval.  Margins cover rounding (n_C is under-estimated).
struct CullRec {
    double ox, oy, oz;   // virtual source
    double tx, ty, tz;   // unit axis
    double slo, shi;     // beam interval in arc length
};

struct Reach {
    double d2, sm2;
    bool ok;
};

__device__ __forceinline__ Reach reach(const CullRec& S, const Patch& p) {
    double vx = p.cx - S.ox, vy = p.cy - S.oy, vz = p.cz - S.oz;
    double sc = vx * S.tx + vy * S.ty + vz * S.tz;
    double vv = vx * vx + vy * vy + vz * vz;
    double nc2 = fmax(vv - sc * sc, 0.0);
    double rad = p.rad * (1.0 + 1e-9) + 1e-6 * (1.0 + fabs(sc));
    double sa = fmax(sc - rad, S.slo), sb = fmin(sc + rad, S.shi);
    double sm = fmax(fabs(sa), fabs(sb));
    double nc = (double)__builtin_amdgcn_sqrtf((float)nc2) * (1.0 - 1e-6);
    double d = fmax(nc - rad, 0.0);
    return Reach{d * d, sm * sm, sa <= sb};
}

__device__ __forceinline__ bool reach_band(const Reach& r, double kap, double kap_eps2) {
    return r.ok & (r.d2 <= fma(kap, r.sm2, kap_eps2) * (1.0 + 1e-9));
}

// A wave-uniform value of lane b of a per-lane double / int64.
__device__ __forceinline__ double lane_f64(double v, int b) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), b);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), b);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ int64_t lane_i64(int64_t v, int b) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), b);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), b);
    return ((int64_t)hi << 32) | (unsigned)lo;
}

// Band constants of one source for the cull: kappa_b and kappa_b eps_b^2.
// Bands<NB> (NB = 1, 4, 8) keeps up to NB bands in wave-uniform registers
// (absent bands get constants that never pass); Bands<0> takes any count up
// to kMaxBands with band b's constants in lane b of a vector register.
template <int NB>
struct Bands {
    double kap[NB], kape[NB];
    __device__ __forceinline__ void load(const JobConst* __restrict__ jobs, int64_t job0, int n_freq, int) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            kap[b] = -1.0;
            kape[b] = -1.0;
            if (b < n_freq) {
                kap[b] = jobs[job0 + b].kappa;
                kape[b] = kap[b] * jobs[job0 + b].eps2;
            }
        }
    }
    __device__ __forceinline__ constexpr int count() const { return NB; }
    __device__ __forceinline__ bool pass(const Reach& r, int b) const { return reach_band(r, kap[b], kape[b]); }
};

template <>
struct Bands<0> {
    double kapv, kapev;
    int n;
    __device__ __forceinline__ void load(const JobConst* __restrict__ jobs, int64_t job0, int n_freq, int lane) {
        n = n_freq;
        kapv = kapev = 0.0;
        if (lane < n_freq) {
            kapv = jobs[job0 + lane].kappa;
            kapev = kapv * jobs[job0 + lane].eps2;
        }
    }
    __device__ __forceinline__ int count() const { return n; }
    __device__ __forceinline__ bool pass(const Reach& r, int b) const {
        return reach_band(r, lane_f64(kapv, b), lane_f64(kapev, b));
    }
};

// Level 0 of the cull: for every chunk of kCullThreads segments of a split
// and every hyper-patch (kHyperSupers consecutive super-patches), a bit per
// segment that may pass for some band.  One workgroup per chunk; mask words
// at ((split * chunks_per_split + chunk) * n_hyper + h) * kWaves + wave.
template <int NB>
__global__ __launch_bounds__(kCullThreads) void k_cull_hyper(const JobConst* __restrict__ jobs,
                                                             const SegRec* __restrict__ rec,
                                                             const Patch* __restrict__ hypers, int n_hyper,
                                                             int n_freq, int chunks_per_split,
                                                             const CullSplit* __restrict__ splits,
                                                             const int32_t* __restrict__ n_splits,
                                                             unsigned long long* __restrict__ hmask,
                                                             const Patch* __restrict__ supers, int n_super,
                                                             int per_super, unsigned* __restrict__ weight) {
    constexpr int kWaves = kCullThreads / kWave;
    if ((int)blockIdx.y >= *n_splits) return;     // the grid covers the most pieces a pass can have
    const CullSplit sl = splits[blockIdx.y];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t j = sl.begin + (int64_t)blockIdx.x * kCullThreads + tid;
    Bands<NB> B;
    B.load(jobs, (int64_t)sl.src * n_freq, n_freq, lane);
    CullRec me{0, 0, 0, 0, 0, 1, 1, 0};
    const bool valid = j < sl.end;
    if (valid) {
        const double2* q = reinterpret_cast<const double2*>(rec + j);
        const double2 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3], a4 = q[4];
        me = CullRec{-0.5 * a0.x, -0.5 * a0.y, -0.5 * a1.x, a2.x, a2.y, a3.x, a4.x, a4.y};
    }
    unsigned long long* out = hmask + ((int64_t)blockIdx.y * chunks_per_split + blockIdx.x) * n_hyper * kWaves;
    for (int h = 0; h < n_hyper; ++h) {
        const Reach r = reach(me, hypers[h]);
        bool any = false;
#pragma unroll
        for (int b = 0; b < B.count(); ++b) any |= B.pass(r, b);
        const unsigned long long bal = __ballot(valid && any);
        if (lane == 0) out[h * kWaves + wv] = bal;
        if (bal == 0ull) continue;
        // the count pass's weights: these segments (per_super = 0: weight of
        // the (piece, hyper-patch)), or those of them that also reach each
        // super-patch of the hyper-patch (level 1's test)
        if (!per_super) {
            if (lane == 0) atomicAdd(weight + (int64_t)blockIdx.y * n_hyper + h, (unsigned)__popcll(bal));
            continue;
        }
        const int q1 = min((h + 1) * kHyperSupers, n_super);
        for (int q = h * kHyperSupers; q < q1; ++q) {
            const Reach rq = reach(me, supers[q]);
            bool in = false;
#pragma unroll
            for (int b = 0; b < B.count(); ++b) in |= B.pass(rq, b);
            const unsigned long long bq = __ballot(valid && any && in);
            if (lane == 0 && bq != 0ull)
                atomicAdd(weight + (int64_t)blockIdx.y * n_super + q, (unsigned)__popcll(bq));
        }
    }
}

// The count pass's launch order: heaviest cull waves first, by the number of
// their piece's segments that reach their super-patch (per_super: weight
// [piece n_super + super-patch]) or else their hyper-patch (weight[piece
// n_hyper + hyper-patch]), 16 classes of its log2, zero last, so that the
// long waves of the super-patches next to a source do not start at the end
// of the grid.  A counting sort in two launches over one thread per wave
// (wave = piece n_super + super-patch): the class sizes (ctr[0, 16)), then
// each block reserves its range of every class (ctr[16, 32)).  The order
// within a class is that of the atomics; the lists do not depend on it.
__device__ __forceinline__ int cull_order_class(unsigned w) {
    return w == 0u ? 15 : max(0, 14 - (31 - __builtin_clz(w)));
}
template <bool SCATTER>
__global__ __launch_bounds__(256) void k_cull_order(const unsigned* __restrict__ weight, int per_super,
                                                    int n_super, int n_hyper, int64_t n_waves,
                                                    unsigned* __restrict__ ctr, int32_t* __restrict__ order) {
    __shared__ unsigned cnt[16], base[16];
    if (threadIdx.x < 16) cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cls = -1;
    unsigned loc = 0u;
    if (i < n_waves) {
        const int64_t piece = i / n_super;
        cls = cull_order_class(per_super ? weight[i]
                                         : weight[piece * n_hyper + (i - piece * n_super) / kHyperSupers]);
        loc = atomicAdd(&cnt[cls], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        const unsigned c = cnt[threadIdx.x];
        if (!SCATTER) {
            if (c != 0u) atomicAdd(&ctr[threadIdx.x], c);
        } else {
            unsigned b = 0u;
            for (int k = 0; k < (int)threadIdx.x; ++k) b += ctr[k];
            base[threadIdx.x] = c != 0u ? b + atomicAdd(&ctr[16 + threadIdx.x], c) : 0u;
        }
    }
    if (!SCATTER) return;
    __syncthreads();
    if (cls >= 0) order[base[cls] + loc] = (int32_t)i;
}

// Cull, levels 1 and 2.  One wave per (super-patch of kSuperPatches
// patches, split of one source's segment range): no workgroup barriers.
// Three queues in LDS, each in segment order, each drained in full batches
// of 64 (a partial batch waits for the next chunk):
//   the split is walked in chunks of 64 segments; the segments that level 0
//   keeps for the super-patch's hyper-patch are queued by index;
//   level 1: a batch of queued segments is loaded (one record per lane) and
//            tested against the super-patch sphere for every band of its
//            source; survivors, with their records and band masks, are queued
//            (the level-2 queue holds one batch in LDS: survivors past it
//            wait in their lanes' registers until that batch is tested);
//   level 2: a batch of survivors is tested against the 16 patches, band by
//            band, and appended to the (job, patch) lists.
// The list cursors of the wave's 16 patches live in LDS between batches and
// in lane b of one register (band b) during a patch's band loop.  The count
// pass leaves one length per (job, patch, split); the fill pass starts every
// cursor at the exclusive prefix sum of those lengths, so each job-patch list
// is the concatenation of its splits in segment order: deterministic, and
// identical between the two passes.
//
// Batch records (up to 8 bands).  The count pass also writes each level-2
// batch it tests as a record: the batch's 64 segment indices and, per (patch
// pm, band b), the ballot of the lanes that passed, at cell pm * NB + b.  A
// wave takes records in blocks of kBatchBlock from one of kBatchRegions
// counters (chosen by a hash of the wave), each over its own range of cap_r
// records (a multiple of kBatchBlock).  A block starts with a header: the
// wave, the number of its records in use, and the wave's list cursor of
// every cell, relative to the wave's first entry, as it stood before the
// block's first batch.  heads[2 wave] is a block of the wave (kChainNone: the
// wave tested no batch; kChainOverflow: it ran out of blocks) and
// heads[2 wave + 1] its number of batches.  A wave whose block does not fit
// stops recording and adds what it still tests to its region's counter, so
// that the counters tell the host what each region needed.  The fill pass
// replays every block of a complete wave on its own (no geometry, no record
// gathers: one load per lane per record, the cursors of the 16 x NB cells in
// lane c of one or two registers) and recomputes only the waves that ran out
// of blocks: either way the same decisions land at the same list positions.
constexpr int kBatchBlock = 4;                             // records a wave takes at a time
constexpr int kBatchRegions = 256;                         // record counters (power of two)
constexpr int kBatchCtrStride = 32;                        // counters 128 bytes apart
constexpr int32_t kChainNone = -1;                         // the wave tested no level-2 batch
constexpr int32_t kChainOverflow = -2;                     // recompute the wave in the fill pass

// A block for C = 16 nb cells (nb = 1, 4 or 8): the header (the wave and the
// records in use as int32, 8 bytes of padding, then the C cursors as int32),
// then kBatchBlock records of 64 segment indices (int32) followed by the
// ballot (uint64) of cell pm * nb + b.  All offsets are multiples of 16.
__host__ __device__ constexpr int64_t batch_hdr_bytes(int cells) { return 16 + 4 * (int64_t)cells; }
__host__ __device__ constexpr int64_t batch_rec_bytes(int cells) { return 4 * kWave + 8 * (int64_t)cells; }
__host__ __device__ constexpr int64_t batch_block_bytes(int cells) {
    return batch_hdr_bytes(cells) + kBatchBlock * batch_rec_bytes(cells);
}
// Bytes per record, the header shared out over a block's records.
size_t cull_batch_bytes(int nb) { return (size_t)batch_block_bytes(kSuperPatches * nb) / kBatchBlock; }
int cull_batch_regions() { return kBatchRegions; }
int cull_batch_ctr_stride() { return kBatchCtrStride; }
int cull_batch_block() { return kBatchBlock; }

// The largest region counter: what the most loaded region needed.
__global__ __launch_bounds__(kBatchRegions) void k_cull_need(const unsigned* __restrict__ ctr,
                                                            unsigned* __restrict__ need) {
    __shared__ unsigned m[kBatchRegions / kWave];
    unsigned v = ctr[threadIdx.x * kBatchCtrStride];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o));
    if ((threadIdx.x & 63) == 0) m[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned r = 0u;
        for (int w = 0; w < kBatchRegions / kWave; ++w) r = max(r, m[w]);
        *need = r;
    }
}

template <bool FILL, int NB>
__global__ __launch_bounds__(kWave) void k_cull(const JobConst* __restrict__ jobs, const SegRec* __restrict__ rec,
                                                const Patch* __restrict__ patches, const Patch* __restrict__ supers,
                                                int n_patch, int n_freq, const int64_t* __restrict__ src_cnt,
                                                const CullSplit* __restrict__ splits,
                                                const int32_t* __restrict__ n_splits,
                                                const unsigned long long* __restrict__ hmask, int n_hyper,
                                                int chunks_per_split, int32_t* __restrict__ counts,
                                                const int64_t* __restrict__ off, int32_t* __restrict__ lists,
                                                unsigned char* __restrict__ bat, unsigned* __restrict__ bat_ctr,
                                                int64_t cap_r, int32_t* __restrict__ heads,
                                                const int32_t* __restrict__ order) {
    constexpr int kQ = 2 * kWave;                         // a partial batch plus one more
    constexpr int kNB = NB > 0 ? NB : kMaxBands;
    __shared__ int32_t q1[kQ];                            // level-1 queue: segment indices
    __shared__ __align__(16) CullRec q_rec[kWave];        // level-2 queue (one batch): records, indices,
    __shared__ int32_t q_seg[kWave];                      // band masks
    __shared__ unsigned long long q_mask[kWave];
    __shared__ int64_t cur_s[kSuperPatches * kNB];        // cursor of (patch pm, band b) at pm * kNB + b
    __shared__ __align__(16) Patch q_patch[kSuperPatches];  // the super-patch's patches
    // this wave: (piece, super-patch) = wave_id / n_super, wave_id % n_super,
    // taken from the launch order when there is one
    const int64_t slot_id = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int64_t wave_id = order ? (int64_t)order[slot_id] : slot_id;
    const int piece = (int)(wave_id / gridDim.x);
    const int sp = (int)(wave_id - (int64_t)piece * gridDim.x);
    // the piece and the super-patch, loaded before the level-0 test so that a
    // wave that goes on does not wait for them after it (piece < the grid's
    // height, the pieces' allocation; those past the last are not used)
    const int n_spl = *n_splits;
    const CullSplit sl = splits[piece];
    const Patch SPt = supers[sp];
    // level-0 bits of 64-segment chunk ci for the super-patch's hyper-patch
    const unsigned long long* hm = hmask + (int64_t)piece * chunks_per_split * n_hyper * 4 +
                                   (int64_t)(sp / kHyperSupers) * 4;
    {
        // most waves have no segment that may reach their hyper-patch: they
        // end here, their counts zero and their chain empty from the pass's
        // set-up (every word of a piece's level 0 is written, zero past its
        // end; those of pieces past the last hold old bits, and those waves
        // end at the piece check)
        const int n_words = chunks_per_split * 4;
        bool any = false;
        for (int cl = threadIdx.x; cl < n_words; cl += kWave)
            any |= hm[(int64_t)(cl >> 2) * n_hyper * 4 + (cl & 3)] != 0ull;
        if (__ballot(any) == 0ull) return;
    }
    if (piece >= n_spl) return;                          // the grid covers the most pieces a pass can have
    const int lane = threadIdx.x;
    const int64_t job0 = (int64_t)sl.src * n_freq;
    const int64_t cnt0 = src_cnt[2 * sl.src], n_piece = src_cnt[2 * sl.src + 1];
    Bands<NB> B;
    B.load(jobs, job0, n_freq, lane);
    const int p0 = sp * kSuperPatches;
    // the 16 patches, read by every level-2 batch: from LDS rather than one
    // scalar load (and wait) per patch and batch
    if (lane < 2 * kSuperPatches) {
        const int p = min(p0 + (lane >> 1), n_patch - 1);
        reinterpret_cast<double2*>(q_patch)[lane] = reinterpret_cast<const double2*>(patches + p)[lane & 1];
    }
    for (int pm = 0; pm < kSuperPatches; ++pm) {
        const int p = p0 + pm;
        if (lane < n_freq)
            cur_s[pm * kNB + lane] =
                (FILL && p < n_patch) ? off[cnt0 + ((int64_t)lane * n_patch + p) * n_piece + sl.idx] : 0;
    }
    wave_lds_fence();
    constexpr int kCells = kSuperPatches * (NB > 0 ? NB : 1);         // cells per record
    constexpr int64_t kBlock = batch_block_bytes(kCells), kHdr = batch_hdr_bytes(kCells);
    constexpr int64_t kRec = batch_rec_bytes(kCells);
    if (FILL && heads[2 * wave_id] != kChainOverflow) return;   // replayed by k_cull_replay, or empty
    // count pass: this wave's current block and the records used in it
    const unsigned region = ((unsigned)wave_id * 0x9E3779B1u) >> 24;
    unsigned* my_ctr = bat_ctr + region * kBatchCtrStride;
    int32_t head = kChainNone;
    int64_t blk = -1;
    int used = kBatchBlock, n_batch = 0, n_lost = 0;
    bool chain_ok = true;
    // level 2 over queue entries [0, n), n <= 64
    auto level2 = [&](int n) __attribute__((always_inline)) {
        const bool valid = lane < n;
        const int i = valid ? lane : 0;
        const CullRec S = q_rec[i];
        const int32_t seg = q_seg[i];
        const unsigned long long bm = valid ? q_mask[i] : 0ull;
        int64_t slot = -1;                                // count pass: this batch's record, if it has one
        if constexpr (!FILL) ++n_batch;
        if constexpr (!FILL && NB > 0) {
            if (chain_ok && used == kBatchBlock) {
                unsigned got = 0u;
                if (lane == 0) got = atomicAdd(my_ctr, (unsigned)kBatchBlock);
                got = __builtin_amdgcn_readfirstlane(got);
                if ((int64_t)got + kBatchBlock <= cap_r) {
                    blk = ((int64_t)region * cap_r + got) / kBatchBlock;
                    if (head == kChainNone) head = (int32_t)blk;
                    // the header: this wave and its cursors before the block
                    wave_lds_fence();
                    int32_t* hd = reinterpret_cast<int32_t*>(bat + blk * kBlock);
                    if (lane == 0) hd[0] = (int32_t)wave_id;
#pragma unroll
                    for (int k = 0; k < (kCells + kWave - 1) / kWave; ++k)
                        if (k * kWave + lane < kCells) hd[4 + k * kWave + lane] = (int32_t)cur_s[k * kWave + lane];
                    used = 0;
                } else {
                    chain_ok = false;
                }
            }
            if (chain_ok) {
                slot = used++;
                if (lane == 0) reinterpret_cast<int32_t*>(bat + blk * kBlock)[1] = used;
            } else {
                ++n_lost;
            }
        }
        unsigned long long mrec[2] = {0ull, 0ull};        // count pass: cell c's ballot in lane c & 63
        for (int pm = 0; pm < kSuperPatches; ++pm) {
            const int p = p0 + pm;
            if (p >= n_patch) break;
            const Reach r = reach(S, q_patch[pm]);
            int64_t cur = lane < n_freq ? cur_s[pm * kNB + lane] : 0;
#pragma unroll
            for (int b = 0; b < B.count(); ++b) {
                const bool k2 = ((bm >> b) & 1ull) & B.pass(r, b);
                const unsigned long long bl = __ballot(k2);
                if (bl == 0ull) continue;
                if (FILL && k2) lists[lane_i64(cur, b) + lanes_before(bl)] = seg;
                cur += lane == b ? (int64_t)__popcll(bl) : 0;
                if constexpr (!FILL && NB > 0) {
                    const int c = pm * NB + b;
                    if (c < kWave) {
                        mrec[0] = lane == c ? bl : mrec[0];
                    } else {
                        mrec[1] = lane == c - kWave ? bl : mrec[1];
                    }
                }
            }
            if (lane < n_freq) cur_s[pm * kNB + lane] = cur;
        }
        if constexpr (!FILL && NB > 0) {
            if (slot >= 0) {
                unsigned char* rp = bat + blk * kBlock + kHdr + slot * kRec;
                reinterpret_cast<int32_t*>(rp)[lane] = valid ? seg : -1;
                unsigned long long* mk = reinterpret_cast<unsigned long long*>(rp + 4 * kWave);
#pragma unroll
                for (int k = 0; k < (kCells + kWave - 1) / kWave; ++k)
                    if (k * kWave + lane < kCells) mk[k * kWave + lane] = mrec[k];
            }
        }
    };
    int qn = 0;                                           // level-2 queue length
    // level 1 over level-1 queue entries [0, n), n <= 64
    auto level1 = [&](int n) __attribute__((always_inline)) {
        const bool valid = lane < n;
        const int32_t j = q1[valid ? lane : 0];
        unsigned long long mask = 0ull;
        CullRec me{0, 0, 0, 0, 0, 1, 1, 0};
        if (valid) {
            const double2* q = reinterpret_cast<const double2*>(rec + j);
            const double2 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3], a4 = q[4];
            me = CullRec{-0.5 * a0.x, -0.5 * a0.y, -0.5 * a1.x, a2.x, a2.y, a3.x, a4.x, a4.y};
            const Reach r = reach(me, SPt);
#pragma unroll
            for (int b = 0; b < B.count(); ++b) mask |= (unsigned long long)B.pass(r, b) << b;
        }
        const unsigned long long bal = __ballot(mask != 0ull);
        if (bal == 0ull) return;
        // survivors at queue positions past the batch keep their records in
        // registers until the full batch has been tested
        const int pos = qn + lanes_before(bal);
        if (mask != 0ull && pos < kWave) {
            q_rec[pos] = me;
            q_seg[pos] = j;
            q_mask[pos] = mask;
        }
        qn += __popcll(bal);
        wave_lds_fence();
        if (qn >= kWave) {
            level2(kWave);
            wave_lds_fence();
            if (mask != 0ull && pos >= kWave) {
                q_rec[pos - kWave] = me;
                q_seg[pos - kWave] = j;
                q_mask[pos - kWave] = mask;
            }
            wave_lds_fence();
            qn -= kWave;
        }
    };
    const int n_chunks = (int)((sl.end - sl.begin + kWave - 1) / kWave);
    int q1n = 0;                                          // level-1 queue length
    // 64 chunks' level-0 words at a time, one per lane; only chunks with a
    // surviving segment are visited
    for (int cb = 0; cb < n_chunks; cb += kWave) {
        const int cl = cb + lane;
        const unsigned long long word = cl < n_chunks ? hm[(int64_t)(cl >> 2) * n_hyper * 4 + (cl & 3)] : 0ull;
        unsigned long long live = __ballot(word != 0ull);
        while (live) {
            const int k = __builtin_ctzll(live);
            live &= live - 1ull;
            const unsigned long long bits = (unsigned long long)lane_i64((int64_t)word, k);
            const int ci = cb + k;
            if ((bits >> lane) & 1ull)
                q1[q1n + lanes_before(bits)] = (int32_t)(sl.begin + (int64_t)ci * kWave + lane);
            q1n += __popcll(bits);
            wave_lds_fence();
            if (q1n >= kWave) {
                level1(kWave);
                const int rest = q1n - kWave;
                const int32_t t = lane < rest ? q1[kWave + lane] : 0;
                wave_lds_fence();
                if (lane < rest) q1[lane] = t;
                wave_lds_fence();
                q1n = rest;
            }
        }
    }
    if (q1n > 0) level1(q1n);
    if (qn > 0) level2(qn);
    if (!FILL) {
        wave_lds_fence();
        for (int pm = 0; pm < kSuperPatches; ++pm) {
            const int p = p0 + pm;
            if (p < n_patch && lane < n_freq)
                counts[cnt0 + ((int64_t)lane * n_patch + p) * n_piece + sl.idx] = (int32_t)cur_s[pm * kNB + lane];
        }
        if constexpr (NB > 0) {
            if (lane == 0) {
                heads[2 * wave_id] = chain_ok ? head : kChainOverflow;
                heads[2 * wave_id + 1] = n_batch;
                if (n_lost > kBatchBlock)      // the failed block's counter step covered the first of them
                    atomicAdd(my_ctr, (unsigned)((n_lost - 1) / kBatchBlock * kBatchBlock));
            }
        } else {
            if (lane == 0) heads[2 * wave_id] = n_batch > 0 ? kChainOverflow : kChainNone;
        }
    }
}

// The fill pass of the waves whose batch records are complete: one wave per
// block of records (grid: blocks x regions; a block's position past what its
// region handed out ends the wave), no LDS.  A block holds its wave, so the
// wave's pieces of the lists start at the prefix sums of the count pass as
// in k_cull, plus the block's own cursors; they live in lane c & 63 of
// cr[c >> 6].  The records are written in order, the next one loaded while
// the current one is written.
template <int NB>
__global__ __launch_bounds__(kWave) void k_cull_replay(const CullSplit* __restrict__ splits, int n_super,
                                                     int n_patch, int n_freq, const int64_t* __restrict__ src_cnt,
                                                     const int64_t* __restrict__ off,
                                                     const unsigned char* __restrict__ bat,
                                                     const unsigned* __restrict__ bat_ctr, int64_t cap_r,
                                                     const int32_t* __restrict__ heads, int32_t* __restrict__ lists) {
    constexpr int kCells = kSuperPatches * NB;
    constexpr int kRegs = (kCells + kWave - 1) / kWave;
    constexpr int64_t kBlock = batch_block_bytes(kCells), kHdr = batch_hdr_bytes(kCells);
    constexpr int64_t kRec = batch_rec_bytes(kCells);
    const int lane = threadIdx.x;
    const int region = blockIdx.y;
    const int64_t handed = min<int64_t>(bat_ctr[region * kBatchCtrStride], cap_r);
    if ((int64_t)blockIdx.x * kBatchBlock >= handed) return;
    const int64_t blk = ((int64_t)region * cap_r) / kBatchBlock + blockIdx.x;
    const unsigned char* bp = bat + blk * kBlock;
    const int32_t* hd = reinterpret_cast<const int32_t*>(bp);
    const int64_t wave_id = __builtin_amdgcn_readfirstlane(hd[0]);
    const int n = __builtin_amdgcn_readfirstlane(hd[1]);
    if (heads[2 * wave_id] == kChainOverflow) return;     // recomputed by k_cull
    const int64_t piece = wave_id / n_super;
    const CullSplit sl = splits[piece];
    const int64_t cnt0 = src_cnt[2 * sl.src], n_piece = src_cnt[2 * sl.src + 1];
    const int p0 = (int)(wave_id - piece * n_super) * kSuperPatches;
    int64_t cr[kRegs];
#pragma unroll
    for (int k = 0; k < kRegs; ++k) {
        const int c = k * kWave + lane, pm = c / NB, b = c % NB;
        cr[k] = c < kCells && p0 + pm < n_patch && b < n_freq
                    ? off[cnt0 + ((int64_t)b * n_patch + p0 + pm) * n_piece + sl.idx] + hd[4 + c] : 0;
    }
    auto load = [&](int j, int32_t& seg, unsigned long long* m) {
        const unsigned char* rp = bp + kHdr + j * kRec;
        seg = reinterpret_cast<const int32_t*>(rp)[lane];
        const unsigned long long* mk = reinterpret_cast<const unsigned long long*>(rp + 4 * kWave);
#pragma unroll
        for (int k = 0; k < kRegs; ++k) m[k] = k * kWave + lane < kCells ? mk[k * kWave + lane] : 0ull;
    };
    // one wait per record: the next record's loads are issued before the
    // current one is written, and settled after its stores
    int32_t seg;
    unsigned long long m[kRegs];
    load(0, seg, m);
    settle(seg);
#pragma unroll
    for (int k = 0; k < kRegs; ++k) settle(m[k]);
    for (int i = 0; i < n; ++i) {
        int32_t seg_n = 0;
        unsigned long long m_n[kRegs];
#pragma unroll
        for (int k = 0; k < kRegs; ++k) m_n[k] = 0ull;
        if (i + 1 < n) load(i + 1, seg_n, m_n);
#pragma unroll
        for (int k = 0; k < kRegs; ++k) {
            unsigned long long live = __ballot(m[k] != 0ull);
            while (live) {
                const int c = __builtin_ctzll(live);
                live &= live - 1ull;
                const unsigned long long bl = (unsigned long long)lane_i64((int64_t)m[k], c);
                if ((bl >> lane) & 1ull) lists[lane_i64(cr[k], c) + lanes_before(bl)] = seg;
            }
            cr[k] += __popcll(m[k]);                      // lane c: cell c's ballot
        }
        settle(seg_n);
#pragma unroll
        for (int k = 0; k < kRegs; ++k) settle(m_n[k]);
        seg = seg_n;
#pragma unroll
        for (int k = 0; k < kRegs; ++k) m[k] = m_n[k];
    }
}

// The counters of item i = (source s, band b) * n_patch + patch p: the
// pieces of source s, at src_cnt[2 s] + (b n_patch + p) src_cnt[2 s + 1].
__device__ __forceinline__ int64_t item_cnt(int64_t i, int n_patch, int n_freq, const int64_t* __restrict__ src_cnt,
                                            int64_t& n_piece) {
    const int64_t job = i / n_patch, p = i - job * n_patch, s = job / n_freq, b = job - s * n_freq;
    n_piece = src_cnt[2 * s + 1];
    return src_cnt[2 * s] + (b * n_patch + p) * n_piece;
}

// Length of every item's list: the span of its pieces in the prefix sum.
__global__ void k_item_lengths(const int64_t* __restrict__ off, int32_t n_items, int n_patch, int n_freq,
                               const int64_t* __restrict__ src_cnt, int32_t* __restrict__ len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    int64_t n_piece;
    const int64_t c = item_cnt(i, n_patch, n_freq, src_cnt, n_piece);
    len[i] = (int32_t)(off[c + n_piece] - off[c]);
}

// ids[i] = i: the payload of the longest-first item sort.
__global__ void k_iota(int32_t* __restrict__ ids, int32_t n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ids[i] = i;
}

// ------------------------------------------------------------- pair kernels
// Beam term of one (segment, receiver) pair without the job's common weight
// k eps / (8 pi^2):
//   B = w Gamma (s + i eps)/(s^2 + eps^2) exp(-(k eps/2) a) exp(2 pi i cyc),
//   a = n^2/den,  den = s^2 + eps^2,  cyc = (f/c) s (1 + a/2).
// The pair kernels read segments from an LDS tile that is staged per work
// unit, so job-dependent per-segment constants are folded in once per tile:
// the gate's c2 - |o|^2 and, in MIX and F32, the complex weight and eps times
// it as FP32.  gate() evaluates the arc length, the gate and the beam
// interval (FP64 in F64 and MIX); term() adds the beam term to (ur, ui), the
// complex rotation fused into the accumulation; the term is exactly zero when
// `live` is false (the Gaussian factor is forced to zero) and finite for any
// input, so the kernel runs it on all lanes of a wave with a passing lane.
struct TileRec {
    double m2ox, m2oy;   // -2 o
    double m2oz, c2oo;   // gate constant of the job minus |o|^2
    double tx, ty;       // unit axis
    double tz, mot;      //   and -o.t
    double slo, shi;     // beam interval in arc length
    double oo, pad;      // |o|^2; isotropic MIX: arg(w Gamma) in cycles
    double wgr, wgi;     // F64: w Gamma.  F32 and anisotropic MIX: float4 (w Gamma, eps w Gamma) as
                         // (Re, Im, Re, Im).  Isotropic MIX: |w Gamma| as FP32 in wgr, f/c in wgi
};
static_assert(sizeof(TileRec) == 112, "TileRec layout");

template <int MODE>
struct Beam;

constexpr int kF64 = 0, kMIX = 1, kF32 = 2;
// Pair-kernel variants: the precision mode, plus kAbsorb when any job has
// atmospheric absorption (without it the term skips the absorption exponent),
// plus kAniso for anisotropic beams.
constexpr int kAbsorb = 4;
constexpr int kAniso = 8;

__device__ __forceinline__ float4 tile_weights(const TileRec& S) {
    return *reinterpret_cast<const float4*>(&S.wgr);
}

template <>
struct Beam<kF64> {
    using T = double;
    struct Geo { double s, l; };   // arc length, |R - o|^2 - |o|^2
    __device__ __forceinline__ static bool gate(const TileRec& S, const JobConst& J, double X, double Y, double Z,
                                                double R2, Geo& g) {
        g.s = fma(X, S.tx, fma(Y, S.ty, fma(Z, S.tz, S.mot)));
        g.l = fma(X, S.m2ox, fma(Y, S.m2oy, fma(Z, S.m2oz, R2)));
        const double rhs = fma(g.s * J.gate_c1, g.s, S.c2oo);
        return g.l <= rhs && g.s >= S.slo && g.s < S.shi;
    }
    template <bool ABS>
    __device__ __forceinline__ static void term(const TileRec& S, const JobConst& J, const Geo& g, bool live,
                                                double& ur, double& ui) {
        const double s = g.s;
        const double n2 = fma(-s, s, g.l + S.oo);
        const double den = fma(s, s, J.eps2);
        const double rden = 1.0 / den;
        const double a = n2 * rden;
        const double cyc = s * fma(J.hfk, a, J.fk);
        const double ph = cyc - floor(cyc);
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double ge = ABS ? fma(s, J.aexp, a * J.gexp) : a * J.gexp;       // Gaussian (and absorption)
        const double w = live ? rden * exp(ge) : 0.0;
        const double cr = fma(s, S.wgr, -J.eps * S.wgi) * w;
        const double ci = fma(s, S.wgi, J.eps * S.wgr) * w;
        ur = fma(cr, cs, fma(-ci, sn, ur));
        ui = fma(cr, sn, fma(ci, cs, ui));
    }
};

// MIX: the gate, the arc length s, the squared normal distance n^2, 1/den
// (FP32 reciprocal and one Newton step), a = n^2/den and the phase in cycles,
// (f/c) s (1 + a/2) + arg(w Gamma)/(2 pi), reduced modulo one, in FP64 (the
// correction (f/2c) s a alone reaches G s / (2 pi eps) cycles at the gate's
// edge, hundreds for narrow beams); the Gaussian, sine and cosine, and the
// amplitude in FP32, with the weight as its modulus times (s + i eps) and its
// argument carried by the phase.
template <>
struct Beam<kMIX> {
    using T = float;
    using Geo = Beam<kF64>::Geo;
    __device__ __forceinline__ static bool gate(const TileRec& S, const JobConst& J, double X, double Y, double Z,
                                                double R2, Geo& g) {
        return Beam<kF64>::gate(S, J, X, Y, Z, R2, g);
    }
    template <bool ABS>
    __device__ __forceinline__ static void term(const TileRec& S, const JobConst& J, const Geo& g, bool live,
                                                float& ur, float& ui) {
        const double s = g.s;
        const double n2 = fma(-s, s, g.l + S.oo);
        const double den = fma(s, s, J.eps2);
        const float r0f = __builtin_amdgcn_rcpf((float)den);
        const double r0 = (double)r0f;
        const double rden = fma(r0, fma(-den, r0, 1.0), r0);                 // one Newton step
        const double a = n2 * rden;
        const float ph = (float)__builtin_amdgcn_fract(fma(s, fma(J.hfk, a, S.wgi), S.pad));   // S.wgi = f/c
        const float sn = __builtin_amdgcn_sinf(ph);                          // sin(2 pi ph)
        const float cs = __builtin_amdgcn_cosf(ph);
        const float sf = (float)s;
        const float gg = (float)a * (float)J.gexp2;                          // Gaussian exponent, base 2
        const float g2 = live ? (ABS ? fmaf(sf, (float)J.aexp2, gg) : gg) : -INFINITY;
        const float w = r0f * __builtin_amdgcn_exp2f(g2) * *reinterpret_cast<const float*>(&S.wgr);
        const float cr = sf * w, ci = (float)J.eps * w;                      // |w Gamma| (s + i eps) / den e^g
        ur = fmaf(cr, cs, fmaf(-ci, sn, ur));
        ui = fmaf(cr, sn, fmaf(ci, cs, ui));
    }
};

template <>
struct Beam<kF32> {
    using T = float;
    struct Geo { float s, n2, den; };
    __device__ __forceinline__ static bool gate(const TileRec& S, const JobConst& J, double Xd, double Yd, double Zd,
                                                double, Geo& g) {
        const float X = (float)Xd, Y = (float)Yd, Z = (float)Zd;
        const float vx = X + 0.5f * (float)S.m2ox, vy = Y + 0.5f * (float)S.m2oy, vz = Z + 0.5f * (float)S.m2oz;
        g.s = vx * (float)S.tx + vy * (float)S.ty + vz * (float)S.tz;
        g.n2 = fmaxf(vx * vx + vy * vy + vz * vz - g.s * g.s, 0.0f);
        g.den = fmaf(g.s, g.s, (float)J.eps2);
        return g.n2 <= (float)J.kappa * g.den && g.s >= (float)S.slo && g.s < (float)S.shi;
    }
    template <bool ABS>
    __device__ __forceinline__ static void term(const TileRec& S, const JobConst& J, const Geo& g, bool live,
                                                float& ur, float& ui) {
        const float rden = __builtin_amdgcn_rcpf(g.den);
        const float cyc = (float)J.fk * fmaf(0.5f * g.n2 * g.s, rden, g.s);
        const float ph = __builtin_amdgcn_fractf(cyc);
        const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
        const float gg = g.n2 * rden * (float)J.gexp2;
        const float w = rden * __builtin_amdgcn_exp2f(live ? (ABS ? fmaf(g.s, (float)J.aexp2, gg) : gg) : -INFINITY);
        const float4 W = tile_weights(S);
        const float cr = fmaf(g.s, W.x, -W.w) * w;
        const float ci = fmaf(g.s, W.y, W.z) * w;
        ur = fmaf(cr, cs, fmaf(-ci, sn, ur));
        ui = fmaf(cr, sn, fmaf(ci, cs, ui));
    }
};

// Anisotropic beams: Eq. (1) with Q = diag(q1, q2), q_m = s - i eps_m, and
// P = I/c (Eq. (2) in a homogeneous medium), in the segment's ray frame
// (e1, e2 = t x e1) from the table (FrameRec; by default e1 = z x t / |z x t|,
// the frame the ground, roofs and walls of the box scenes transport); only
// n1^2 and n2^2 enter.  With
//   n1 = (R - o).e1,  n2^2 = n^2 - n1^2,  den_m = s^2 + eps_m^2,  a_m = n_m^2/den_m:
//   Gaussian exp(-(k/2)(eps a1 + epsb a2)), kept iff eps a1 + epsb a2 <= 2G/k,
//   phase (f/c) s (1 + (a1 + a2)/2) cycles,
//   i sqrt(q01/q1) sqrt(q02/q2) = sqrt(eps epsb / (den1 den2)) / (2 sqrt(b1 b2))
//                                 * (s (b1 + b2) + i (b1 b2 - s^2)),  b_m = sqrt(den_m) + eps_m
// (the product of the principal roots sqrt(eps_m - i s) = (r_m, -s/(2 r_m)),
// r_m^2 = b_m/2: every eps_m - i s has a positive real part, so the principal
// branch is the continuous one along the beam).  The job weight is k/(8 pi^2).
// gate() is the isotropic pre-gate on the envelope of the two widths (it keeps
// every pair the exact gate keeps); term() applies the exact gate and returns
// its decision.
struct TileRecA {
    TileRec b;           // isotropic record; b.pad holds -o.e1
    double e1x, e1y;     // frame vector e1
    double e1z, pad;
};
static_assert(sizeof(TileRecA) == 144, "TileRecA layout");

// 1/d from the FP32 reciprocal and one Newton step in FP64.
__device__ __forceinline__ double rcp_newton(double d) {
    const double r0 = (double)__builtin_amdgcn_rcpf((float)d);
    return fma(r0, fma(-d, r0, 1.0), r0);
}

struct GeoA {
    double s, l;         // as Beam<kF64>::Geo
    double x, y, z;      // receiver (for n1)
};

template <int MODE>
struct BeamA;

template <>
struct BeamA<kMIX> {
    using T = float;
    using Geo = GeoA;
    __device__ __forceinline__ static bool gate(const TileRecA& S, const JobConst& J, double X, double Y, double Z,
                                                double R2, Geo& g) {
        Beam<kF64>::Geo h;
        const bool k = Beam<kF64>::gate(S.b, J, X, Y, Z, R2, h);
        g.s = h.s;
        g.l = h.l;
        g.x = X;
        g.y = Y;
        g.z = Z;
        return k;
    }
    template <bool ABS>
    __device__ __forceinline__ static bool term(const TileRecA& S, const JobConst& J, const Geo& g, bool live,
                                                float& ur, float& ui) {
        const double s = g.s;
        const double nn = fma(-s, s, g.l + S.b.oo);                      // n1^2 + n2^2
        const double n1 = fma(g.x, S.e1x, fma(g.y, S.e1y, fma(g.z, S.e1z, S.b.pad)));     // offset along e1
        const double q1 = n1 * n1;
        const double q2 = nn - q1;                                       // offset^2 along e2
        const double den1 = fma(s, s, J.epsa2), den2 = fma(s, s, J.epsb2);
        const double a1 = q1 * rcp_newton(den1), a2 = q2 * rcp_newton(den2);
        const double e = fma(J.eps, a1, J.epsb * a2);
        const bool in = live && e <= J.gate_a;
        const double cyc = s * fma(J.hfk, a1 + a2, J.fk);                // phase in cycles, FP64
        const float ph = (float)__builtin_amdgcn_fract(cyc);
        const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
        const float sf = (float)s;
        const float gg = (float)(e * J.gexpa2);
        const float w = __builtin_amdgcn_exp2f(in ? (ABS ? fmaf(sf, (float)J.aexp2, gg) : gg) : -INFINITY);
        const float d1f = (float)den1, d2f = (float)den2;
        const float d1 = __builtin_amdgcn_sqrtf(d1f), d2 = __builtin_amdgcn_sqrtf(d2f);
        const float e1 = (float)J.eps, e2 = (float)J.epsb;
        const float b1 = d1 + e1, b2 = d2 + e2;
        const float ss = sf * sf;
        // b1 b2 - s^2 = (s^2 (eps^2 + epsb^2) + eps^2 epsb^2) / (d1 d2 + s^2) + eps d2 + epsb d1 + eps epsb
        // (no cancellation when s >> eps)
        const float x = fmaf(ss, (float)(J.epsa2 + J.epsb2), (float)(J.epsa2 * J.epsb2)) *
                        __builtin_amdgcn_rcpf(fmaf(d1, d2, ss));
        const float im = x + fmaf(e1, d2, fmaf(e2, d1, e1 * e2));
        const float re = sf * (b1 + b2);
        const float pre = (float)J.ampc * __builtin_amdgcn_rsqf(d1f * d2f * (b1 * b2)) * w;
        const float4 W = tile_weights(S.b);
        const float cr = (re * W.x - im * W.y) * pre;
        const float ci = (re * W.y + im * W.x) * pre;
        ur = fmaf(cr, cs, fmaf(-ci, sn, ur));
        ui = fmaf(cr, sn, fmaf(ci, cs, ui));
        return in;
    }
};

template <>
struct BeamA<kF64> {
    using T = double;
    using Geo = GeoA;
    __device__ __forceinline__ static bool gate(const TileRecA& S, const JobConst& J, double X, double Y, double Z,
                                                double R2, Geo& g) {
        return BeamA<kMIX>::gate(S, J, X, Y, Z, R2, g);
    }
    template <bool ABS>
    __device__ __forceinline__ static bool term(const TileRecA& S, const JobConst& J, const Geo& g, bool live,
                                                double& ur, double& ui) {
        const double s = g.s;
        const double nn = fma(-s, s, g.l + S.b.oo);
        const double n1 = fma(g.x, S.e1x, fma(g.y, S.e1y, fma(g.z, S.e1z, S.b.pad)));
        const double q1 = n1 * n1;
        const double q2 = nn - q1;
        const double den1 = fma(s, s, J.epsa2), den2 = fma(s, s, J.epsb2);
        const double a1 = q1 / den1, a2 = q2 / den2;
        const double e = fma(J.eps, a1, J.epsb * a2);
        const bool in = live && e <= J.gate_a;
        const double cyc = s * fma(J.hfk, a1 + a2, J.fk);
        const double ph = cyc - floor(cyc);
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double ge = ABS ? fma(s, J.aexp, e * J.gexpa) : e * J.gexpa;
        const double w = in ? exp(ge) : 0.0;
        const double d1 = sqrt(den1), d2 = sqrt(den2);
        const double b1 = d1 + J.eps, b2 = d2 + J.epsb;
        const double bb = b1 * b2;
        const double re = s * (b1 + b2);
        const double im = fma(-s, s, bb);
        const double pre = J.ampc / sqrt(den1 * den2 * bb) * w;
        const double cr = (re * S.b.wgr - im * S.b.wgi) * pre;
        const double ci = (re * S.b.wgi + im * S.b.wgr) * pre;
        ur = fma(cr, cs, fma(-ci, sn, ur));
        ui = fma(cr, sn, fma(ci, cs, ui));
        return in;
    }
};

template <>
struct BeamA<kF32> {
    using T = float;
    struct Geo { float s, n2, x, y, z; };
    __device__ __forceinline__ static bool gate(const TileRecA& S, const JobConst& J, double X, double Y, double Z,
                                                double R2, Geo& g) {
        Beam<kF32>::Geo h;
        const bool k = Beam<kF32>::gate(S.b, J, X, Y, Z, R2, h);
        g.s = h.s;
        g.n2 = h.n2;
        g.x = (float)X;
        g.y = (float)Y;
        g.z = (float)Z;
        return k;
    }
    template <bool ABS>
    __device__ __forceinline__ static bool term(const TileRecA& S, const JobConst& J, const Geo& g, bool live,
                                                float& ur, float& ui) {
        const float s = g.s;
        const float n1 = fmaf(g.x, (float)S.e1x, fmaf(g.y, (float)S.e1y, fmaf(g.z, (float)S.e1z, (float)S.b.pad)));
        const float q1 = n1 * n1;
        const float q2 = fmaxf(g.n2 - q1, 0.0f);
        const float e1 = (float)J.eps, e2 = (float)J.epsb;
        const float den1 = fmaf(s, s, (float)J.epsa2), den2 = fmaf(s, s, (float)J.epsb2);
        const float a1 = q1 * __builtin_amdgcn_rcpf(den1), a2 = q2 * __builtin_amdgcn_rcpf(den2);
        const float e = fmaf(e1, a1, e2 * a2);
        const bool in = live && e <= (float)J.gate_a;
        const float cyc = (float)J.fk * fmaf(0.5f * s, a1 + a2, s);
        const float ph = __builtin_amdgcn_fractf(cyc);
        const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
        const float gg = e * (float)J.gexpa2;
        const float w = __builtin_amdgcn_exp2f(in ? (ABS ? fmaf(s, (float)J.aexp2, gg) : gg) : -INFINITY);
        const float d1 = __builtin_amdgcn_sqrtf(den1), d2 = __builtin_amdgcn_sqrtf(den2);
        const float b1 = d1 + e1, b2 = d2 + e2;
        const float ss = s * s;
        const float x = fmaf(ss, (float)(J.epsa2 + J.epsb2), (float)(J.epsa2 * J.epsb2)) *
                        __builtin_amdgcn_rcpf(fmaf(d1, d2, ss));
        const float im = x + fmaf(e1, d2, fmaf(e2, d1, e1 * e2));
        const float re = s * (b1 + b2);
        const float pre = (float)J.ampc * __builtin_amdgcn_rsqf(den1 * den2 * (b1 * b2)) * w;
        const float4 W = tile_weights(S.b);
        const float cr = (re * W.x - im * W.y) * pre;
        const float ci = (re * W.y + im * W.x) * pre;
        ur = fmaf(cr, cs, fmaf(-ci, sn, ur));
        ui = fmaf(cr, sn, fmaf(ci, cs, ui));
        return in;
    }
};

// The pair-kernel variants whose tile records carry the weight in polar form.
template <int MODE>
constexpr bool kPolar = (MODE & 3) == kMIX && (MODE & kAniso) == 0;

// The beam model and LDS tile record of a pair-kernel variant.
template <int MODE>
using BeamOf = typename std::conditional<(MODE & kAniso) != 0, BeamA<MODE & 3>, Beam<MODE & 3>>::type;
template <int MODE>
using TileOf = typename std::conditional<(MODE & kAniso) != 0, TileRecA, TileRec>::type;

// One segment for one receiver: wave-uniform skip when no lane passes.  The
// term is added to (fr, fi), accumulators in the term's precision that the
// kernel adds into its FP64 sums once per tile.
template <int MODE>
__device__ __forceinline__ int pair_one(const TileOf<MODE>& S, const JobConst& J, double X, double Y, double Z,
                                        double R2, typename BeamOf<MODE>::T& fr, typename BeamOf<MODE>::T& fi) {
    using B = BeamOf<MODE>;
    constexpr bool ABS = (MODE & kAbsorb) != 0;
    typename B::Geo g;
    const bool k0 = B::gate(S, J, X, Y, Z, R2, g);
    if (__ballot(k0) == 0ull) return 0;
    branch_barrier();
    if constexpr ((MODE & kAniso) != 0) {
        return (int)B::template term<ABS>(S, J, g, k0, fr, fi);
    } else {
        B::template term<ABS>(S, J, g, k0, fr, fi);
        return (int)k0;
    }
}

// Two consecutive segments for one receiver: their beam terms are independent
// dependency chains (each into its own accumulators) that the compiler
// interleaves; one wave-uniform branch skips both when no lane passes either
// gate.
template <int MODE>
__device__ __forceinline__ int pair_two(const TileOf<MODE>& S0, const TileOf<MODE>& S1, const JobConst& J, double X,
                                        double Y, double Z, double R2, typename BeamOf<MODE>::T* fr,
                                        typename BeamOf<MODE>::T* fi) {
    using B = BeamOf<MODE>;
    constexpr bool ABS = (MODE & kAbsorb) != 0;
    typename B::Geo g0, g1;
    const bool k0 = B::gate(S0, J, X, Y, Z, R2, g0);
    const bool k1 = B::gate(S1, J, X, Y, Z, R2, g1);
    if (__ballot(k0 || k1) == 0ull) return 0;
    branch_barrier();
    if constexpr ((MODE & kAniso) != 0) {
        const bool h0 = B::template term<ABS>(S0, J, g0, k0, fr[0], fi[0]);
        const bool h1 = B::template term<ABS>(S1, J, g1, k1, fr[1], fi[1]);
        return (int)h0 + (int)h1;
    } else {
        B::template term<ABS>(S0, J, g0, k0, fr[0], fi[0]);
        B::template term<ABS>(S1, J, g1, k1, fr[1], fi[1]);
        return (int)k0 + (int)k1;
    }
}

// A segment record in registers, as seven named 16-byte vectors (kept out of
// arrays so the compiler keeps them in VGPRs): vector loads, 128-bit LDS stores.
#define GBS_REC_REGS(n) double2 n##0, n##1, n##2, n##3, n##4, n##5, n##6
#define GBS_REC_LOAD(n, recp, j)                                                  \
    do {                                                                          \
        const double2* p_ = reinterpret_cast<const double2*>((recp) + (j));       \
        n##0 = p_[0]; n##1 = p_[1]; n##2 = p_[2];                                 \
        n##3 = p_[3]; n##4 = p_[4]; n##5 = p_[5]; n##6 = p_[6];                   \
    } while (0)

// Builds a lane's tile record from its segment record (seven 16-byte vectors
// in SegRec field order) for job J and stores it to the wave's LDS tile.
// POLAR (the isotropic MIX pair kernel): the weight in polar form, its phase
// in cycles in the spare slot and its modulus as FP32 in place of the complex
// weight, followed by the job's f/c (so the phase's FMAs read both of their
// job constants from different register files).
template <int MODE, bool POLAR = false>
__device__ __forceinline__ void stage_rec(TileRec* dst, double2 r0, double2 r1, double2 r2, double2 r3, double2 r4,
                                          double2 r5, double2 r6, const JobConst& J) {
    double2* q = reinterpret_cast<double2*>(dst);
    q[0] = r0;
    q[1] = make_double2(r1.x, J.gate_c2 - r1.y);
    q[2] = r2;
    q[3] = r3;
    q[4] = r4;
    q[5] = make_double2(r1.y, POLAR ? r6.x : 0.0);
    if (POLAR) {
        union { float2 f; double d; } m;
        m.f = make_float2((float)hypot(r5.x, r5.y), 0.f);
        q[6] = make_double2(m.d, J.fk);
    } else if (MODE == kF64) {
        q[6] = r5;
    } else {
        *reinterpret_cast<float4*>(q + 6) =
            make_float4((float)r5.x, (float)r5.y, (float)(J.eps * r5.x), (float)(J.eps * r5.y));
    }
}
// The anisotropic tile record: the isotropic one plus the frame vector e1 of
// the segment (f0 = (e1x, e1y), f1 = (e1z, -o.e1) of its FrameRec), with -o.e1
// in the isotropic record's spare slot.
template <int MODE>
__device__ __forceinline__ void stage_rec_a(TileRecA* dst, double2 r0, double2 r1, double2 r2, double2 r3,
                                            double2 r4, double2 r5, double2 r6, double2 f0, double2 f1,
                                            const JobConst& J) {
    stage_rec<MODE>(&dst->b, r0, r1, r2, r3, r4, r5, r6, J);
    dst->b.pad = f1.y;
    double2* q = reinterpret_cast<double2*>(&dst->e1x);
    q[0] = f0;
    q[1] = make_double2(f1.x, 0.0);
}
#define GBS_STAGE(MODE, dst, n, J) stage_rec<MODE>((dst), n##0, n##1, n##2, n##3, n##4, n##5, n##6, (J))
#define GBS_STAGE_P(MODE, POLAR, dst, n, J) \
    stage_rec<MODE, POLAR>((dst), n##0, n##1, n##2, n##3, n##4, n##5, n##6, (J))
#define GBS_STAGE_A(MODE, dst, n, J) \
    stage_rec_a<MODE>((dst), n##0, n##1, n##2, n##3, n##4, n##5, n##6, n##f0, n##f1, (J))

// Pops the next work item (wave-uniform) from the global counter.  Lane 0
// issues the atomic.  Callers put branch_barrier() in front of it and issue
// their own end-of-item atomics from lane kLastLane: if both ends of the loop
// body were guarded by the same lane predicate, the compiler could thread the
// two guards across the back edge and re-run the index shuffle without lane 0.
__device__ __forceinline__ int pop_item(unsigned* ctr) {
    int it = 0;
    if ((threadIdx.x & (kWave - 1)) == 0) it = (int)atomicAdd(ctr, 1u);
    it = __shfl(it, 0);
    return __builtin_amdgcn_readfirstlane(it);
}
constexpr int kLastLane = kWave - 1;

// Persistent forward kernel: one wavefront per work unit, a chunk of at most
// a fixed number of segments of one (job, patch) list (long lists - patches
// next to a source see nearly every beam - are spread over many waves); the
// patch holds 64 * NR receivers, lane l owns receivers l, l + 64, ...
// The item's segment list is walked in tiles of 64: lane l gathers record l
// of the next tile with vector loads (one memory round trip per tile, issued
// a whole tile ahead), the tile goes to the wave's LDS slice, and every
// segment is then read back as a wave-uniform LDS broadcast.
// P (job-major, original receiver order) accumulates scale * sum.
#ifndef GBS_PAIR_MIN_WAVES
#define GBS_PAIR_MIN_WAVES 1
#endif
template <int MODE, int NR, bool COUNT>
__global__ __launch_bounds__(kPairThreads, GBS_PAIR_MIN_WAVES) void k_pairs(const JobConst* __restrict__ jobs,
                                              const Work* __restrict__ work, const int32_t* __restrict__ n_work_p,
                                              int32_t n_patch, unsigned* __restrict__ ctr,
                                              const int32_t* __restrict__ lists, const SegRec* __restrict__ rec,
                                              const FrameRec* __restrict__ frames,
                                              const double* __restrict__ rx, const double* __restrict__ ry,
                                              const double* __restrict__ rz, const double* __restrict__ r2,
                                              double* __restrict__ partial, unsigned long long* __restrict__ n_active) {
    constexpr bool kA = (MODE & kAniso) != 0;
    using Tile = TileOf<MODE>;
    using T = typename BeamOf<MODE>::T;
    __shared__ __align__(16) Tile tile[kPairThreads / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    Tile* const my = tile[threadIdx.x / kWave];
    const int n_work = __builtin_amdgcn_readfirstlane(*n_work_p);
    unsigned long long active = 0;
    for (;;) {
        branch_barrier();
        const int w = pop_item(ctr);
        if (w >= n_work) break;
        const int item = __builtin_amdgcn_readfirstlane(work[w].item);
        const int64_t beg = work[w].beg, end = work[w].end;
        const int job = item / n_patch, patch = item - job * n_patch;
        const JobConst J = jobs[job];
        double X[NR], Y[NR], Z[NR], R2[NR], ar[NR], ai[NR];
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            const int64_t i = (int64_t)patch * (64 * NR) + 64 * m + lane;
            X[m] = rx[i];
            Y[m] = ry[i];
            Z[m] = rz[i];
            R2[m] = r2[i];
            ar[m] = 0.0;
            ai[m] = 0.0;
        }
        // indices run two tiles ahead of the records they address, records one
        // tile ahead of the tile being evaluated (clamped: the tail re-reads a
        // valid entry, never out of range)
        GBS_REC_REGS(nx);
        double2 nxf0 = make_double2(0.0, 0.0), nxf1 = nxf0;   // frame (anisotropic beams)
        const int32_t idx_first = lists[min(beg + lane, end - 1)];
        GBS_REC_LOAD(nx, rec, idx_first);
        if constexpr (kA) {
            const double2* f_ = reinterpret_cast<const double2*>(frames + idx_first);
            nxf0 = f_[0];
            nxf1 = f_[1];
        }
        int32_t idx_ahead = lists[min(beg + kWave + lane, end - 1)];
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int cnt = (int)min<int64_t>(kWave, end - e0);
            wave_lds_fence();
            if constexpr (kA) {
                GBS_STAGE_A((MODE & 3), my + lane, nx, J);
            } else {
                GBS_STAGE_P((MODE & 3), kPolar<MODE>, my + lane, nx, J);
            }
            wave_lds_fence();
            GBS_REC_LOAD(nx, rec, idx_ahead);
            if constexpr (kA) {
                const double2* f_ = reinterpret_cast<const double2*>(frames + idx_ahead);
                nxf0 = f_[0];
                nxf1 = f_[1];
            }
            idx_ahead = lists[min(e0 + 2 * kWave + lane, end - 1)];
            // the tile's terms in the term precision (FP32 in MIX: at most 64
            // terms per sum), then once into the FP64 sums
            T fr[NR][2], fi[NR][2];
#pragma unroll
            for (int m = 0; m < NR; ++m) fr[m][0] = fr[m][1] = fi[m][0] = fi[m][1] = T(0);
            int k = 0;
#ifndef GBS_PAIR_SINGLE
            for (; k + 2 <= cnt; k += 2) {
                const Tile S0 = my[k], S1 = my[k + 1];
#pragma unroll
                for (int m = 0; m < NR; ++m) {
                    const int hit = pair_two<MODE>(S0, S1, J, X[m], Y[m], Z[m], R2[m], fr[m], fi[m]);
                    if (COUNT) active += (unsigned long long)hit;
                }
            }
#endif
            for (; k < cnt; ++k) {
                const Tile S = my[k];
#pragma unroll
                for (int m = 0; m < NR; ++m) {
                    const int hit = pair_one<MODE>(S, J, X[m], Y[m], Z[m], R2[m], fr[m][0], fi[m][0]);
                    if (COUNT) active += (unsigned long long)hit;
                }
            }
#pragma unroll
            for (int m = 0; m < NR; ++m) {
                ar[m] += (double)fr[m][0] + (double)fr[m][1];
                ai[m] += (double)fi[m][0] + (double)fi[m][1];
            }
        }
#pragma unroll
        for (int m = 0; m < NR; ++m) {
            double* p = partial + 2 * (((int64_t)w * NR + m) * kWave + lane);
            p[0] = ar[m];
            p[1] = ai[m];
        }
    }
    if (COUNT) {
        double tot = wave_sum_last((double)active);
        if (lane == kLastLane) atomicAdd(n_active, (unsigned long long)tot);
    }
}

// Work units per item, in the longest-first item order: ceil(len / chunk).
__global__ void k_work_counts(const int32_t* __restrict__ order, const int32_t* __restrict__ len, int32_t n_items,
                              int32_t chunk, int32_t* __restrict__ nwork) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n_items) return;
    nwork[k] = k < n_items ? (len[order[k]] + chunk - 1) / chunk : 0;
}

// Lays out the work units of every item from the exclusive scan of the counts.
__global__ void k_make_work(const int32_t* __restrict__ order, const int64_t* __restrict__ off, int n_patch,
                            int n_freq, const int64_t* __restrict__ src_cnt,
                            const int32_t* __restrict__ wbase, int32_t n_items, int32_t chunk,
                            Work* __restrict__ work, int32_t* __restrict__ item_wbase,
                            int32_t* __restrict__ item_wcount, int32_t* __restrict__ n_work) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_items) return;
    const int item = order[k];
    int64_t n_piece;
    const int64_t c = item_cnt(item, n_patch, n_freq, src_cnt, n_piece);
    const int64_t beg = off[c], end = off[c + n_piece];
    const int32_t b = wbase[k], cnt = wbase[k + 1] - b;
    for (int c = 0; c < cnt; ++c) {
        Work u;
        u.beg = beg + (int64_t)c * chunk;
        u.end = min(u.beg + chunk, end);
        u.item = item;
        u.pad = 0;
        work[b + c] = u;
    }
    item_wbase[item] = b;
    item_wcount[item] = cnt;
    if (k == n_items - 1) *n_work = b + cnt;
}

// P[job][receiver] += scale * (sum of the item's work-unit partials, in
// unit order).  One thread per (item, receiver slot).
__global__ void k_reduce_partials(const JobConst* __restrict__ jobs, const int32_t* __restrict__ item_wbase,
                                  const int32_t* __restrict__ item_wcount, int32_t n_items, int32_t n_patch, int nr,
                                  const int32_t* __restrict__ perm, int64_t n_rcv, const double* __restrict__ partial,
                                  double* __restrict__ P, double* __restrict__ TL, int write) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int per = kWave * nr;
    if (t >= (int64_t)n_items * per) return;
    const int item = (int)(t / per), slot = (int)(t - (int64_t)item * per);
    const int cnt = item_wcount[item];
    if (cnt == 0 && !write) return;
    const int job = item / n_patch, patch = item - job * n_patch;
    const int m = slot / kWave, lane = slot - m * kWave;
    const int32_t o = perm[(int64_t)patch * per + slot];
    if (o < 0) return;
    const int64_t base = item_wbase[item];
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < cnt; ++c) {
        const double* p = partial + 2 * (((base + c) * nr + m) * kWave + lane);
        sr += p[0];
        si += p[1];
    }
    const int64_t out = (int64_t)job * n_rcv + o;
    double* q = P + 2 * out;
    const double sc = jobs[job].scale;
    if (write) {
        // a call's only pass: every (job, receiver) output is written here,
        // with its TL
        const double pr = sc * sr, pi = sc * si;
        q[0] = pr;
        q[1] = pi;
        if (TL) {
            const double mag = hypot(pr, pi);
            TL[out] = mag > 0.0 ? -20.0 * log10(mag) : INFINITY;
        }
    } else {
        q[0] += sc * sr;
        q[1] += sc * si;
    }
}

// TL = -20 log10 |P|  (+inf where P = 0).
__global__ void k_tl(const double* __restrict__ P, int64_t n, double* __restrict__ TL) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double m = hypot(P[2 * i], P[2 * i + 1]);
    TL[i] = m > 0.0 ? -20.0 * log10(m) : INFINITY;
}

// ----------------------------------------------------------------- adjoint
// Adjoint pair terms.  With u = scale * wG * B (forward term) and the
// convention dL = Re sum lambda dP:
//   d ln u/dR   = t (ik - 1/q - (ik/2) n^2/q^2 - alpha) + (ik/q) nvec,  nvec = R - o - s t
//   (alpha: the atmospheric absorption of the job, exp(-alpha s) in u)
//   d ln u/deps = 1/eps + i/q - (k/2) n^2/q^2
//   dP/dGamma_f = scale * sum_j d(prod Gamma_j)/dGamma_f * w_j * B_j
// With 1/q = (s + i eps) rden and 1/q^2 = (s^2 - eps^2 + 2 i eps s) rden^2.
template <typename T>
struct AdjTerms {
    T Br, Bi;        // B / (w prod Gamma): beam term without weight and coefficients
    T ctr, cti;      // coefficient of t in d ln u/dR
    T cnr, cni;      // coefficient of nvec
    T der, dei;      // d ln u/deps
};

template <typename T, bool ABS>
__device__ __forceinline__ void adj_factors(T s, T n2, T rden, T eps, T k, T aexp, AdjTerms<T>& A) {
    T r2d = rden * rden;
    T iq_r = s * rden, iq_i = eps * rden;                              // 1/q
    T iq2_r = (s * s - eps * eps) * r2d, iq2_i = 2 * eps * s * r2d;    // 1/q^2
    T hk = (T)0.5 * k * n2;
    // ik - 1/q - (ik/2) n^2/q^2 - alpha : (ik/2)n^2/q^2 = hk*(i*iq2_r - iq2_i)
    A.ctr = -iq_r + hk * iq2_i;
    if (ABS) A.ctr += aexp;
    A.cti = k - iq_i - hk * iq2_r;
    // ik/q = i k (iq_r + i iq_i) = -k iq_i + i k iq_r
    A.cnr = -k * iq_i;
    A.cni = k * iq_r;
    // 1/eps + i/q - (k/2) n^2/q^2 ; i/q = -iq_i + i iq_r
    A.der = (T)1 / eps - iq_i - hk * iq2_r;
    A.dei = iq_r - hk * iq2_i;
}

// Receiver gradient of one pair: gt t + gn nvec with nvec = R - o - s t
// = (gt - gn s) t + gn R + gn (-2 o) / 2.  Per receiver the kernel sums
// V = sum (gt - gn s) t, W = sum gn (-2 o) and G = sum gn, and writes
// dL/dR = V + W / 2 + G R once per work unit: 7 FMAs per pair instead of
// forming nvec (the cancellation costs about two of FP64's 16 digits).
struct AdjAcc {
    double vx, vy, vz, wx, wy, wz, g, e;   // V, W, G and dL/deps
};

template <int MODE, typename ST>
__device__ __forceinline__ bool adj_eval(const TileRec& S, const JobConst& J, double X, double Y, double Z, double R2,
                                         ST lr, ST li, AdjAcc& acc, ST& Sr, ST& Si) {
    constexpr bool ABS = (MODE & kAbsorb) != 0;
    Beam<kF64>::Geo g;
    const bool keep = Beam<kF64>::gate(S, J, X, Y, Z, R2, g);
    if (__ballot(keep) == 0ull) return false;    // wave-uniform skip
    branch_barrier();
    if (!keep) return false;
    const double s = g.s;
    const double n2 = fma(-s, s, g.l + S.oo);
    const double den = fma(s, s, J.eps2);
    double rden;
    float r0f = 0.f;
    if ((MODE & 3) == kF64) {
        rden = 1.0 / den;
    } else {
        r0f = __builtin_amdgcn_rcpf((float)den);
        const double r0 = (double)r0f;
        rden = fma(r0, fma(-den, r0, 1.0), r0);                    // one Newton step
    }
    const double a = n2 * rden;
    const double cyc = s * fma(J.hfk, a, J.fk);
    double gt, gn;
    if ((MODE & 3) == kF64) {
        const double ph = cyc - floor(cyc);
        double sn, cs;
        sincospi(2.0 * ph, &sn, &cs);
        const double w = rden * exp(ABS ? fma(s, J.aexp, a * J.gexp) : a * J.gexp);
        AdjTerms<double> A;
        adj_factors<double, ABS>(s, n2, rden, J.eps, J.k, J.aexp, A);
        const double br = s * w, bi = J.eps * w;                  // (s + i eps) rden e^g
        A.Br = br * cs - bi * sn;
        A.Bi = br * sn + bi * cs;
        const double ur = S.wgr * A.Br - S.wgi * A.Bi, ui = S.wgr * A.Bi + S.wgi * A.Br;
        const double vr = lr * ur - li * ui, vi = lr * ui + li * ur;    // lambda u
        gt = vr * A.ctr - vi * A.cti;
        gn = vr * A.cnr - vi * A.cni;
        acc.e += vr * A.der - vi * A.dei;
        Sr += lr * A.Br - li * A.Bi;
        Si += lr * A.Bi + li * A.Br;
    } else {
        const float ph = (float)__builtin_amdgcn_fract(cyc);
        const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
        const float sf = (float)s, epsf = (float)J.eps, kf = (float)J.k;
        const float gg = (float)(a * J.gexp2);
        const float w = r0f * __builtin_amdgcn_exp2f(ABS ? fmaf(sf, (float)J.aexp2, gg) : gg);
        // adj_factors with its shared products: with t1 = Im(1/q) + (k/2) n^2 Re(1/q^2),
        // Im(d ln u/dR . t) = k - t1 and Re(d ln u/deps) = 1/eps - t1; Re(d ln u/dR . t)
        // = -Im(d ln u/deps) (+ the absorption term); the n coefficient is i k (1/q)
        const float r2d = r0f * r0f;
        const float iq_r = sf * r0f, iq_i = epsf * r0f;                          // 1/q
        const float iq2_r = fmaf(sf, sf, -(float)J.eps2) * r2d;                   // Re 1/q^2
        const float iq2_i = (2.0f * epsf) * sf * r2d;                             // Im 1/q^2
        const float hk = (0.5f * kf) * (float)n2;
        const float t1 = fmaf(hk, iq2_r, iq_i);
        const float dei = fmaf(-hk, iq2_i, iq_r);
        const float cti = kf - t1, der = 1.0f / epsf - t1;
        const float ctr = ABS ? (float)J.aexp - dei : -dei;
        const float br = sf * w, bi = epsf * w;
        const float Br = br * cs - bi * sn, Bi = br * sn + bi * cs;
        // lambda B (the coefficient sums), then lambda w Gamma B
        const float lbr = lr * Br - li * Bi, lbi = lr * Bi + li * Br;
        Sr += lbr;
        Si += lbi;
        const float4 Wg = tile_weights(S);                       // (w Gamma, eps w Gamma) as FP32
        const float vr = Wg.x * lbr - Wg.y * lbi, vi = Wg.x * lbi + Wg.y * lbr;
        const float gtf = vr * ctr - vi * cti;
        const float gnf = -kf * fmaf(vr, iq_i, vi * iq_r);       // vr Re(ik/q) - vi Im(ik/q)
        const double c = (double)fmaf(-gnf, sf, gtf);            // gt - gn s
        gn = (double)gnf;
        acc.e += (double)(vr * der - vi * dei);
        acc.vx = fma(c, S.tx, acc.vx);
        acc.vy = fma(c, S.ty, acc.vy);
        acc.vz = fma(c, S.tz, acc.vz);
        acc.wx = fma(gn, S.m2ox, acc.wx);
        acc.wy = fma(gn, S.m2oy, acc.wy);
        acc.wz = fma(gn, S.m2oz, acc.wz);
        acc.g += gn;
        return true;
    }
    const double c = fma(-gn, s, gt);
    acc.vx = fma(c, S.tx, acc.vx);
    acc.vy = fma(c, S.ty, acc.vy);
    acc.vz = fma(c, S.tz, acc.vz);
    acc.wx = fma(gn, S.m2ox, acc.wx);
    acc.wy = fma(gn, S.m2oy, acc.wy);
    acc.wz = fma(gn, S.m2oz, acc.wz);
    acc.g += gn;
    return true;
}

// Anisotropic adjoint (Eq. (1) with Q = diag(q1, q2)).  With n_m the
// offsets along the frame vectors, 1/q_m = (s + i eps_m)/den_m and
// n_m^2/q_m^2 = n_m^2 (s^2 - eps_m^2 + 2 i eps_m s)/den_m^2:
//   d ln u/dR     = t (ik - (1/q1 + 1/q2)/2 - (ik/2)(n1^2/q1^2 + n2^2/q2^2) - alpha)
//                   + (ik n1/q1) e1 + (ik n2/q2) e2
//   d ln u/deps_m = (1/eps_m + i/q_m)/2 - (k/2) n_m^2/q_m^2
// and the coefficient sums take B = u/(scale w prod Gamma) as for isotropic
// beams.  The tile record adds the whole frame.
struct TileRecAdj {
    TileRec b;               // isotropic record; b.pad holds -o.e1
    double e1x, e1y, e1z, moe2;
    double e2x, e2y, e2z, pad;
};
static_assert(sizeof(TileRecAdj) == 176, "TileRecAdj layout");

template <int MODE>
__device__ __forceinline__ void stage_rec_adj(TileRecAdj* dst, double2 r0, double2 r1, double2 r2, double2 r3,
                                              double2 r4, double2 r5, double2 r6, double2 f0, double2 f1,
                                              double2 f2, double2 f3, const JobConst& J) {
    stage_rec<MODE>(&dst->b, r0, r1, r2, r3, r4, r5, r6, J);
    dst->b.pad = f1.y;
    double2* q = reinterpret_cast<double2*>(&dst->e1x);
    q[0] = f0;
    q[1] = make_double2(f1.x, f3.y);
    q[2] = f2;
    q[3] = make_double2(f3.x, 0.0);
}

struct AdjAccA {
    double x, y, z, e1, e2;   // dL/dR and the two beam-parameter sums
};

template <int MODE, typename ST>
__device__ __forceinline__ bool adj_eval_aniso(const TileRecAdj& S, const JobConst& J, double X, double Y, double Z,
                                               double R2, ST lr, ST li, AdjAccA& acc, ST& Sr, ST& Si) {
    constexpr bool ABS = (MODE & kAbsorb) != 0;
    constexpr bool F64 = (MODE & 3) == kF64;
    using T = ST;
    Beam<kF64>::Geo g;
    const bool keep = Beam<kF64>::gate(S.b, J, X, Y, Z, R2, g);    // envelope pre-gate
    if (__ballot(keep) == 0ull) return false;                        // wave-uniform skip
    branch_barrier();
    if (!keep) return false;
    const double s = g.s;
    const double nn = fma(-s, s, g.l + S.b.oo);
    const double n1 = fma(X, S.e1x, fma(Y, S.e1y, fma(Z, S.e1z, S.b.pad)));
    const double n2 = fma(X, S.e2x, fma(Y, S.e2y, fma(Z, S.e2z, S.moe2)));
    const double q1 = n1 * n1, q2 = nn - q1;                         // as the forward's exact gate
    const double den1 = fma(s, s, J.epsa2), den2 = fma(s, s, J.epsb2);
    const double rd1 = F64 ? 1.0 / den1 : rcp_newton(den1), rd2 = F64 ? 1.0 / den2 : rcp_newton(den2);
    const double a1 = q1 * rd1, a2 = q2 * rd2;
    const double e = fma(J.eps, a1, J.epsb * a2);
    if (!(e <= J.gate_a)) return false;
    const double cyc = s * fma(J.hfk, a1 + a2, J.fk);
    T sn, cs, w;
    if constexpr (F64) {
        const double ph = cyc - floor(cyc);
        sincospi(2.0 * ph, &sn, &cs);
        w = exp(ABS ? fma(s, J.aexp, e * J.gexpa) : e * J.gexpa);
    } else {
        const float ph = (float)__builtin_amdgcn_fract(cyc);
        sn = __builtin_amdgcn_sinf(ph);
        cs = __builtin_amdgcn_cosf(ph);
        const float gg = (float)(e * J.gexpa2);
        w = __builtin_amdgcn_exp2f(ABS ? fmaf((float)s, (float)J.aexp2, gg) : gg);
    }
    // B = i sqrt(q01/q1) sqrt(q02/q2) e^{i phase} e^{g}
    const T st = (T)s, e1 = (T)J.eps, e2 = (T)J.epsb, k = (T)J.k;
    const T d1 = sqrt((T)den1), d2 = sqrt((T)den2);
    const T b1 = d1 + e1, b2 = d2 + e2;
    const T re = st * (b1 + b2), im = b1 * b2 - st * st;
    const T pre = (T)J.ampc / sqrt((T)den1 * (T)den2 * (b1 * b2)) * w;
    const T ar = re * pre, ai = im * pre;
    const T Br = ar * cs - ai * sn, Bi = ar * sn + ai * cs;
    T wr, wi;
    if constexpr (F64) {
        wr = S.b.wgr;
        wi = S.b.wgi;
    } else {
        const float4 W = tile_weights(S.b);
        wr = W.x;
        wi = W.y;
    }
    const T ur = wr * Br - wi * Bi, ui = wr * Bi + wi * Br;
    const T vr = lr * ur - li * ui, vi = lr * ui + li * ur;           // lambda u
    const T r1 = (T)rd1, r2 = (T)rd2, m1 = (T)n1, m2 = (T)n2;
    const T n1s = m1 * m1, n2s = m2 * m2;
    const T A1 = n1s * (st * st - e1 * e1) * r1 * r1, B1 = n1s * (2 * e1 * st) * r1 * r1;   // n1^2/q1^2
    const T A2 = n2s * (st * st - e2 * e2) * r2 * r2, B2 = n2s * (2 * e2 * st) * r2 * r2;
    const T hk = (T)0.5 * k;
    T ctr = (T)-0.5 * st * (r1 + r2) + hk * (B1 + B2);
    if (ABS) ctr += (T)J.aexp;
    const T cti = k - (T)0.5 * (e1 * r1 + e2 * r2) - hk * (A1 + A2);
    const T c1r = -k * m1 * e1 * r1, c1i = k * m1 * st * r1;
    const T c2r = -k * m2 * e2 * r2, c2i = k * m2 * st * r2;
    const T gt = vr * ctr - vi * cti, g1 = vr * c1r - vi * c1i, g2 = vr * c2r - vi * c2i;
    const T de1r = (T)0.5 * ((T)1 / e1 - e1 * r1) - hk * A1, de1i = (T)0.5 * st * r1 - hk * B1;
    const T de2r = (T)0.5 * ((T)1 / e2 - e2 * r2) - hk * A2, de2i = (T)0.5 * st * r2 - hk * B2;
    acc.e1 += (double)(vr * de1r - vi * de1i);
    acc.e2 += (double)(vr * de2r - vi * de2i);
    const double Gt = (double)gt, G1 = (double)g1, G2 = (double)g2;
    acc.x = fma(Gt, S.b.tx, fma(G1, S.e1x, fma(G2, S.e2x, acc.x)));
    acc.y = fma(Gt, S.b.ty, fma(G1, S.e1y, fma(G2, S.e2y, acc.y)));
    acc.z = fma(Gt, S.b.tz, fma(G1, S.e1z, fma(G2, S.e2z, acc.z)));
    Sr += lr * Br - li * Bi;
    Si += lr * Bi + li * Br;
    return true;
}

// Persistent adjoint kernel over the same work units as the forward, with
// the same LDS-staged segment tiles.  Per receiver (lane): dL/dR accumulates
// in FP64 and is written as the unit's partial (k_reduce_adjoint adds a
// patch's units in order); per segment: the sum over lanes of lambda * B
// (a reduction within each row of 16 lanes, the four row sums left in the
// tile's LDS slot of the segment) goes to Sseg as an exact fixed-point sum
// (scale fixed_scales[0]) at the end of the tile, one segment per lane; per unit: dL/deps (and dL/deps_e2 for
// anisotropic beams) from wave reductions, reduced per job in unit order by
// k_reduce_eps.  Every output is bitwise repeatable.
template <int MODE>
__global__ __launch_bounds__(kPairThreads) void k_adjoint(const JobConst* __restrict__ jobs,
                                                const Work* __restrict__ work, const int32_t* __restrict__ n_work_p,
                                                int32_t n_patch, unsigned* __restrict__ ctr,
                                                const int32_t* __restrict__ lists, const SegRec* __restrict__ rec,
                                                const FrameRec* __restrict__ frames,
                                                const double* __restrict__ rx, const double* __restrict__ ry,
                                                const double* __restrict__ rz, const double* __restrict__ r2,
                                                const int32_t* __restrict__ perm, int64_t n_rcv,
                                                const double* __restrict__ lambda, double* __restrict__ partial,
                                                const int32_t* __restrict__ seg_perm, Fixed* __restrict__ Sseg,
                                                const double* __restrict__ fixed_scales,
                                                double* __restrict__ eps_partial, double* __restrict__ eps2_partial) {
    constexpr bool kA = (MODE & kAniso) != 0;
    using Tile = typename std::conditional<kA, TileRecAdj, TileRec>::type;
    using Acc = typename std::conditional<kA, AdjAccA, AdjAcc>::type;
    using ST = typename Beam<MODE & 3>::T;                // beam-term precision
    __shared__ __align__(16) Tile tile[kPairThreads / kWave][kWave];
    __shared__ int32_t tile_idx[kPairThreads / kWave][kWave];
    __shared__ ST tile_sum[kPairThreads / kWave][kWave][8];    // per tile segment: row sums of lambda B
    const int lane = threadIdx.x & (kWave - 1);
    Tile* const my = tile[threadIdx.x / kWave];
    int32_t* const my_idx = tile_idx[threadIdx.x / kWave];
    ST (*const my_sum)[8] = tile_sum[threadIdx.x / kWave];
    const int n_work = __builtin_amdgcn_readfirstlane(*n_work_p);
    const double sscale = fixed_scales[0];
    for (;;) {
        branch_barrier();
        const int w = pop_item(ctr);
        if (w >= n_work) break;
        const int item = __builtin_amdgcn_readfirstlane(work[w].item);
        const int64_t beg = work[w].beg, end = work[w].end;
        const int job = item / n_patch, patch = item - job * n_patch;
        const JobConst J = jobs[job];
        const int64_t i = (int64_t)patch * 64 + lane;
        const double X = rx[i], Y = ry[i], Z = rz[i], R2 = r2[i];
        const int32_t o = perm[i];
        ST lr = 0, li = 0;
        if (o >= 0) {
            lr = (ST)lambda[2 * ((int64_t)job * n_rcv + o)];
            li = (ST)lambda[2 * ((int64_t)job * n_rcv + o) + 1];
        }
        Acc acc{};
        GBS_REC_REGS(nx);
        double2 nxf0 = make_double2(0.0, 0.0), nxf1 = nxf0, nxf2 = nxf0, nxf3 = nxf0;
        int32_t idx_cur = lists[min(beg + lane, end - 1)];
        GBS_REC_LOAD(nx, rec, idx_cur);
        if constexpr (kA) {
            const double2* f_ = reinterpret_cast<const double2*>(frames + idx_cur);
            nxf0 = f_[0];
            nxf1 = f_[1];
            nxf2 = f_[2];
            nxf3 = f_[3];
        }
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int cnt = (int)min<int64_t>(kWave, end - e0);
            wave_lds_fence();
            if constexpr (kA) {
                stage_rec_adj<MODE & 3>(my + lane, nx0, nx1, nx2, nx3, nx4, nx5, nx6, nxf0, nxf1, nxf2, nxf3, J);
            } else {
                GBS_STAGE((MODE & 3), my + lane, nx, J);
            }
            my_idx[lane] = seg_perm ? seg_perm[idx_cur] : idx_cur;   // table order for the segment sums
#pragma unroll
            for (int q = 0; q < 8; ++q) my_sum[lane][q] = 0;
            wave_lds_fence();
            idx_cur = lists[min(e0 + kWave + lane, end - 1)];
            GBS_REC_LOAD(nx, rec, idx_cur);
            if constexpr (kA) {
                const double2* f_ = reinterpret_cast<const double2*>(frames + idx_cur);
                nxf0 = f_[0];
                nxf1 = f_[1];
                nxf2 = f_[2];
                nxf3 = f_[3];
            }
            for (int k = 0; k < cnt; ++k) {
                const Tile S = my[k];
                ST Sr = 0, Si = 0;
                bool hit;
                if constexpr (kA) {
                    hit = adj_eval_aniso<MODE>(S, J, X, Y, Z, R2, lr, li, acc, Sr, Si);
                } else {
                    hit = adj_eval<MODE>(S, J, X, Y, Z, R2, lr, li, acc, Sr, Si);
                }
                if (__ballot(hit) != 0ull) {
                    Sr = row_sum_last(Sr);
                    Si = row_sum_last(Si);
                    if ((lane & 15) == 15) {
                        my_sum[k][2 * (lane >> 4)] = Sr;
                        my_sum[k][2 * (lane >> 4) + 1] = Si;
                    }
                }
            }
            // the tile's segment sums, one segment per lane (rows added in order)
            wave_lds_fence();
            const ST tr = (my_sum[lane][0] + my_sum[lane][2]) + (my_sum[lane][4] + my_sum[lane][6]);
            const ST ti = (my_sum[lane][1] + my_sum[lane][3]) + (my_sum[lane][5] + my_sum[lane][7]);
            if (lane < cnt && (tr != 0 || ti != 0)) {
                const int64_t j = my_idx[lane];
                fixed_add(&Sseg[2 * j], J.scale * (double)tr, sscale);
                fixed_add(&Sseg[2 * j + 1], J.scale * (double)ti, sscale);
            }
        }
        double* p = partial + 3 * ((int64_t)w * kWave + lane);
        if constexpr (kA) {
            p[0] = acc.x;
            p[1] = acc.y;
            p[2] = acc.z;
            const double dE1 = wave_sum_last(acc.e1), dE2 = wave_sum_last(acc.e2);
            if (lane == kLastLane) {
                eps_partial[w] = J.scale * dE1;
                eps2_partial[w] = J.scale * dE2;
            }
        } else {
            p[0] = fma(acc.g, X, fma(0.5, acc.wx, acc.vx));
            p[1] = fma(acc.g, Y, fma(0.5, acc.wy, acc.vy));
            p[2] = fma(acc.g, Z, fma(0.5, acc.wz, acc.vz));
            const double dE = wave_sum_last(acc.e);
            if (lane == kLastLane) eps_partial[w] = J.scale * dE;
        }
    }
}

// dR_job[job][receiver] += scale * (sum of the item's unit partials, in unit
// order).  One thread per (item, lane) of 64-receiver patches.
__global__ void k_reduce_adjoint(const JobConst* __restrict__ jobs, const int32_t* __restrict__ item_wbase,
                                 const int32_t* __restrict__ item_wcount, int32_t n_items, int32_t n_patch,
                                 const int32_t* __restrict__ perm, int64_t n_rcv, const double* __restrict__ partial,
                                 double* __restrict__ dR_job) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_items * kWave) return;
    const int item = (int)(t / kWave), lane = (int)(t - (int64_t)item * kWave);
    const int cnt = item_wcount[item];
    if (cnt == 0) return;
    const int job = item / n_patch, patch = item - job * n_patch;
    const int32_t o = perm[(int64_t)patch * kWave + lane];
    if (o < 0) return;
    const int64_t base = item_wbase[item];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int c = 0; c < cnt; ++c) {
        const double* p = partial + 3 * ((base + c) * kWave + lane);
        sx += p[0];
        sy += p[1];
        sz += p[2];
    }
    double* d = dR_job + 3 * ((int64_t)job * n_rcv + o);
    const double sc = jobs[job].scale;
    d[0] += sc * sx;
    d[1] += sc * sy;
    d[2] += sc * sz;
}

// dR[r] = sum over jobs of dR_job[job][r]  (fixed order).
__global__ void k_sum_jobs(const double* __restrict__ dR_job, int32_t n_jobs, int64_t n_rcv, double* __restrict__ dR) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 3 * n_rcv) return;
    double s = 0.0;
    for (int32_t j = 0; j < n_jobs; ++j) s += dR_job[(int64_t)j * 3 * n_rcv + i];
    dR[i] = s;
}

// Z_f += d(prod Gamma_j)/dGamma_f * w_j * S_j for every distinct face f in
// segment j's history (product of the other factors, summed over the
// occurrences of f), as an exact fixed-point sum (scale fixed_scales[1]).
// One thread per segment; the wave walks history positions in step and adds
// the contributions of lanes that hit the same face with one wave reduction
// and one pair of integer atomics per distinct face (most segments of a scene
// share a few faces, the ground above all).  Histories were checked by
// k_records; ids outside [0, n_faces) are skipped.
__global__ void k_face_scatter(int64_t n_segs, const int64_t* __restrict__ face_ptr, int64_t face_base,
                               const int32_t* __restrict__ face_ids, int32_t n_faces, const double* __restrict__ gamma,
                               const double* __restrict__ ray_w, const int32_t* __restrict__ seg_ray,
                               const Fixed* __restrict__ Sseg, const double* __restrict__ fixed_scales,
                               Fixed* __restrict__ Zf) {
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const double zscale = fixed_scales[1], sinv = fixed_scales[2];
    double sr = 0.0, si = 0.0, w = 0.0;
    int64_t b = 0, e = 0;
    if (j < n_segs) {
        sr = fixed_value(Sseg[2 * j], sinv);
        si = fixed_value(Sseg[2 * j + 1], sinv);
        const int64_t f0 = face_ptr[j] - face_base, f1 = face_ptr[j + 1] - face_base;
        if ((sr != 0.0 || si != 0.0) && f0 >= 0 && f1 >= f0) {
            b = f0;
            e = f1;
            w = ray_w[seg_ray[j]];
        }
    }
    const int len = (int)(e - b);
    int max_len = len;
    for (int o = 32; o > 0; o >>= 1) max_len = max(max_len, __shfl_xor(max_len, o));
    for (int l = 0; l < max_len; ++l) {
        int32_t f = -1;
        double zr = 0.0, zi = 0.0;
        if (l < len) {
            f = face_ids[b + l];
            bool skip = f < 0 || f >= n_faces;
            for (int64_t m = b; m < b + l; ++m) skip |= face_ids[m] == f;   // counted at its first occurrence
            if (skip) {
                f = -1;
            } else {
                double dr = 0.0, di = 0.0;
                for (int64_t l2 = b + l; l2 < e; ++l2) {
                    if (face_ids[l2] != f) continue;
                    double pr = 1.0, pi = 0.0;
                    for (int64_t m = b; m < e; ++m) {
                        const int32_t g = face_ids[m];
                        if (m == l2 || g < 0 || g >= n_faces) continue;
                        const double xr = gamma[2 * g], xi = gamma[2 * g + 1];
                        const double nr = pr * xr - pi * xi;
                        pi = pr * xi + pi * xr;
                        pr = nr;
                    }
                    dr += pr;
                    di += pi;
                }
                zr = w * (dr * sr - di * si);
                zi = w * (dr * si + di * sr);
            }
        }
        unsigned long long pending = __ballot(f >= 0);
        while (pending) {
            const int leader = __builtin_ctzll(pending);
            const int32_t f0 = __builtin_amdgcn_readlane(f, leader);
            const bool mine = f == f0;
            const double tr = wave_sum_last(mine ? zr : 0.0), ti = wave_sum_last(mine ? zi : 0.0);
            if (lane == kLastLane) {
                fixed_add(&Zf[2 * (int64_t)f0], tr, zscale);
                fixed_add(&Zf[2 * (int64_t)f0 + 1], ti, zscale);
            }
            pending &= ~__ballot(mine);
        }
    }
}

// Sum over the receivers of |Re lambda| + |Im lambda| per job (a bound on
// sum |lambda|) in a fixed order: one workgroup per (job, piece of the
// receivers) writes a partial sum, k_lambda_l1_sum adds a job's pieces in order;
// also flags non-finite lambda.
__global__ __launch_bounds__(256) void k_lambda_l1(const double* __restrict__ lambda, int64_t n_rcv,
                                                   double* __restrict__ part, int* __restrict__ status) {
    __shared__ double sm[256];
    const int job = blockIdx.x, piece = blockIdx.y, pieces = gridDim.y;
    const int64_t span = (n_rcv + pieces - 1) / pieces;
    const int64_t r0 = piece * span, r1 = min(n_rcv, r0 + span);
    const double* lj = lambda + 2 * (int64_t)job * n_rcv;
    double acc = 0.0;
    bool ok = true;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
        const double x = lj[2 * r], y = lj[2 * r + 1];
        ok &= isfinite(x) && isfinite(y);
        acc += fabs(x) + fabs(y);
    }
    if (!ok) atomicOr(status, kBadLambda);
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)job * pieces + piece] = sm[0];
}

// l1[job] = sum of the job's partial sums (pieces per job), in order.
__global__ void k_lambda_l1_sum(const double* __restrict__ part, int32_t n_jobs, int pieces,
                                double* __restrict__ l1) {
    const int job = blockIdx.x * blockDim.x + threadIdx.x;
    if (job >= n_jobs) return;
    double acc = 0.0;
    for (int c = 0; c < pieces; ++c) acc += part[(int64_t)job * pieces + c];
    l1[job] = acc;
}

// Scales of the adjoint's exact sums.  Segment sums: every contribution is
// scale_job * lambda * B with |B| <= 1/eps (isotropic; scale = k eps/(8 pi^2))
// or <= 1 (anisotropic; scale = k/(8 pi^2)), so sum_job k/(8 pi^2) sum|lambda|,
// doubled against FP32 rounding, bounds every partial sum.  Face sums: at most
// n_segs terms, each |w d(prod Gamma)/dGamma_f S_j| <= bmax * bound_S.
// out = {2^K_S, 2^K_Z, 2^-K_S, 2^-K_Z}.
__global__ void k_fixed_scales(const JobConst* __restrict__ jobs, const double* __restrict__ l1, int32_t n_jobs,
                               int64_t n_segs, const unsigned long long* __restrict__ bmax,
                               double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double bs = 0.0;
    for (int32_t j = 0; j < n_jobs; ++j) bs += jobs[j].k * (1.0 / (8.0 * 3.14159265358979323846 * 3.14159265358979323846)) * l1[j];
    bs *= 2.0;
    const double bz = bs * (double)n_segs * __longlong_as_double((long long)*bmax) * 2.0;
    out[0] = fixed_scale_for(bs);
    out[1] = fixed_scale_for(bz);
    out[2] = 1.0 / out[0];
    out[3] = 1.0 / out[1];
}

// d_eps[job] += sum over the job's work units of eps_partial, in (patch, unit)
// order: one workgroup per job, a strided pass then a fixed tree.
__global__ __launch_bounds__(256) void k_reduce_eps(const int32_t* __restrict__ item_wbase,
                                                    const int32_t* __restrict__ item_wcount, int32_t n_patch,
                                                    const double* __restrict__ eps_partial, double* __restrict__ d_eps) {
    __shared__ double sm[256];
    const int job = blockIdx.x;
    double acc = 0.0;
    for (int p = threadIdx.x; p < n_patch; p += 256) {
        const int item = job * n_patch + p;
        const int b = item_wbase[item], c = item_wcount[item];
        for (int u = 0; u < c; ++u) acc += eps_partial[b + u];
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) d_eps[job] += sm[0];
}

// Zf (FP64) += the pass's exact face sums.
__global__ void k_fixed_flush(const Fixed* __restrict__ acc, int64_t n, const double* __restrict__ fixed_scales,
                              double* __restrict__ out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] += fixed_value(acc[i], fixed_scales[3]);
}

// d_gamma = (Re Z, -Im Z).
__global__ void k_dgamma(const double* __restrict__ Zf, int32_t n_faces, double* __restrict__ d_gamma) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_faces) return;
    d_gamma[2 * i] = Zf[2 * i];
    d_gamma[2 * i + 1] = -Zf[2 * i + 1];
}

// Explicit instantiations used by the host planner.
#define GBS_INST_CULL(F, NB)                                                                                   \
    template __global__ void k_cull<F, NB>(const JobConst*, const SegRec*, const Patch*, const Patch*, int, int,      \
                                           const int64_t*,                                                         \
                                           const CullSplit*, const int32_t*, const unsigned long long*, int, int,    \
                                           int32_t*, const int64_t*, int32_t*, unsigned char*, unsigned*, int64_t,   \
                                           int32_t*, const int32_t*);
#define GBS_INST_CULL_NB(NB)                                                                                   \
    GBS_INST_CULL(false, NB)                                                                                   \
    GBS_INST_CULL(true, NB)                                                                                    \
    template __global__ void k_cull_hyper<NB>(const JobConst*, const SegRec*, const Patch*, int, int, int,       \
                                              const CullSplit*, const int32_t*, unsigned long long*, const Patch*, \
                                              int, int, unsigned*);
GBS_INST_CULL_NB(1)
GBS_INST_CULL_NB(4)
GBS_INST_CULL_NB(8)
GBS_INST_CULL_NB(0)
template __global__ void k_cull_order<false>(const unsigned*, int, int, int, int64_t, unsigned*, int32_t*);
template __global__ void k_cull_order<true>(const unsigned*, int, int, int, int64_t, unsigned*, int32_t*);
#define GBS_INST_REPLAY(NB)                                                                                    \
    template __global__ void k_cull_replay<NB>(const CullSplit*, int, int, int, const int64_t*, const int64_t*, \
                                               const unsigned char*, const unsigned*, int64_t, const int32_t*,  \
                                               int32_t*);
GBS_INST_REPLAY(1)
GBS_INST_REPLAY(4)
GBS_INST_REPLAY(8)
#define GBS_INST_PAIRS(M, N, C)                                                                                  \
    template __global__ void k_pairs<M, N, C>(const JobConst*, const Work*, const int32_t*, int32_t, unsigned*,    \
                                              const int32_t*, const SegRec*, const FrameRec*, const double*,     \
                                              const double*, const double*, const double*, double*,              \
                                              unsigned long long*);
#define GBS_INST_PAIRS_MODE(M) \
    GBS_INST_PAIRS(M, 1, false) GBS_INST_PAIRS(M, 2, false) GBS_INST_PAIRS(M, 4, false) \
    GBS_INST_PAIRS(M, 1, true) GBS_INST_PAIRS(M, 2, true) GBS_INST_PAIRS(M, 4, true)
GBS_INST_PAIRS_MODE(0)
GBS_INST_PAIRS_MODE(1)
GBS_INST_PAIRS_MODE(2)
GBS_INST_PAIRS_MODE(4)
GBS_INST_PAIRS_MODE(5)
GBS_INST_PAIRS_MODE(6)
GBS_INST_PAIRS_MODE(8)
GBS_INST_PAIRS_MODE(9)
GBS_INST_PAIRS_MODE(10)
GBS_INST_PAIRS_MODE(12)
GBS_INST_PAIRS_MODE(13)
GBS_INST_PAIRS_MODE(14)
#define GBS_INST_ADJ(M)                                                                                          \
    template __global__ void k_adjoint<M>(const JobConst*, const Work*, const int32_t*, int32_t, unsigned*,       \
                                          const int32_t*, const SegRec*, const FrameRec*, const double*,          \
                                          const double*, const double*, const double*, const int32_t*, int64_t,   \
                                          const double*, double*, const int32_t*, Fixed*, const double*, double*, \
                                          double*);
GBS_INST_ADJ(0)
GBS_INST_ADJ(1)
GBS_INST_ADJ(4)
GBS_INST_ADJ(5)
GBS_INST_ADJ(8)
GBS_INST_ADJ(9)
GBS_INST_ADJ(12)
GBS_INST_ADJ(13)

}  // namespace gbs

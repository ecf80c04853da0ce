// Internal layout shared by the host planner and the gfx950 kernels of libgbs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbs {

constexpr int kWave = 64;             // CDNA wavefront width
constexpr int kCullThreads = 256;     // cull kernel workgroup (4 waves)
constexpr int kSuperPatches = 16;     // patches per culling super-patch
constexpr int kHyperSupers = 16;      // super-patches per culling hyper-patch (level 0)
constexpr int kPairThreads = 256;     // pair/adjoint workgroup: 4 independent persistent waves
constexpr int kMaxBands = 64;         // bands per call (one bit each in the cull's band masks)

// Per-job constants (job = (source, band)), computed on the host.
struct JobConst {
    int64_t seg_begin;   // segment range of the job's source inside the current pass
    int64_t seg_end;
    double k;            // wavenumber 2 pi f / c
    double eps;          // beam parameter (Rayleigh range) of this job
    double eps2;         // eps^2
    double gate_c1;      // pair kept iff |R-o|^2 <= s^2 * gate_c1 + gate_c2
    double gate_c2;      //   (c1 = 1 + 2G/(k eps), c2 = 2 G eps^2 / (k eps))
    double kappa;        // 2G/(k eps): normal-distance gate n^2 <= kappa (s^2 + eps^2)
    double fk;           // f / c: cycles per metre of travel
    double hfk;          // f / (2c)
    double gexp2;        // -(k eps / 2) log2(e): Gaussian exponent in base 2 per n^2/den
    double gexp;         // -(k eps / 2)
    double scale;        // k eps / (8 pi^2) (anisotropic: k / (8 pi^2)): weight factored out of the sum
    double aexp;         // -alpha: atmospheric absorption exponent per metre of arc length
    double aexp2;        // -alpha log2(e)
    // Anisotropic beams (beam parameter eps along the frame vector e1, epsb
    // along e2).  The cull and the pre-gate then use the envelope of the two
    // widths: kappa = 2G/(k min(eps, epsb)), eps2 = eps epsb (so that
    // kappa eps2 = 2G max(eps, epsb)/k), gate_c1 = 1 + kappa, gate_c2 = kappa eps2.
    double epsb;         // beam parameter along e2
    double epsa2;        // eps^2
    double epsb2;        // epsb^2
    double gate_a;       // exact gate: eps a1 + epsb a2 <= 2G/k
    double gexpa;        // -(k/2): Gaussian exponent per (eps a1 + epsb a2)
    double gexpa2;       // -(k/2) log2(e)
    double ampc;         // sqrt(eps epsb) / 2
    int32_t src;
    int32_t band;
};

// One beam segment, prepared for the pair kernel (job independent).  The
// axis is re-anchored at the virtual source o = a - s0 t, so that the arc
// length of the projection of R is s = R.t - o.t and |R - o|^2 - s^2 = n^2.
struct SegRec {
    double m2ox, m2oy, m2oz;  // -2 o
    double oo;                // |o|^2
    double tx, ty, tz;        // unit axis
    double mot;               // -o.t
    double slo, shi;          // beam interval in arc length [s0 + lo, s0 + hi)
    double wgr, wgi;          // ray solid angle times the reflection-coefficient product
    double wph, pad;          // the weight's argument / (2 pi) (cycles)
};
static_assert(sizeof(SegRec) == 112, "SegRec layout");

// The ray frame of a segment for anisotropic beams (job independent): unit
// vectors e1 and e2 = t x e1 normal to the axis, with -o.e1 and -o.e2, so that
// the offsets of R along them are R.e1 - o.e1 and R.e2 - o.e2.
struct FrameRec {
    double e1x, e1y, e1z, moe1;
    double e2x, e2y, e2z, moe2;
};
static_assert(sizeof(FrameRec) == 64, "FrameRec layout");

struct Patch {
    double cx, cy, cz, rad;   // bounding sphere of a receiver patch
};

// One unit of pair-kernel work: a chunk [beg, end) of one item's list.
struct Work {
    int64_t beg, end;         // range in the concatenated lists
    int32_t item;             // job * n_patch + patch
    int32_t pad;
};
constexpr int kWorkChunk = 2048;      // segments per work unit (bounds the longest unit)

// A contiguous piece of one source's segments, culled by one workgroup.
struct CullSplit {
    int64_t begin, end;       // segment range (pass-local indices)
    int32_t src;              // source of every segment in the range
    int32_t idx;              // index of the piece within its source
};

// Table and receiver checks done by the kernels that read the data anyway:
// each problem sets one bit of a device status word, which the host reads at
// its next synchronisation (before any pair kernel runs) and reports as
// GBS_E_INVALID.  Kernels never read outside an array because of bad data.
enum StatusBit : int {
    kBadSegment = 1,      // non-finite a, s0, lo or hi; lo > hi; |t| != 1
    kBadFacePtr = 2,      // face_ptr not non-decreasing inside [0, face_ptr[n_segs]]
    kBadFaceId = 4,       // face id outside [0, n_faces)
    kBadRayPtr = 8,       // ray_ptr not a CSR over the segments, or a segment without a ray
    kBadRayWeight = 16,   // non-finite or negative ray weight
    kBadReceiver = 32,    // non-finite receiver coordinate
    kBadRaySource = 64,   // ray_src outside [0, n_src) or not non-decreasing
    kBadLambda = 128,     // non-finite adjoint weight lambda
    kBadJob = 256         // frequency, beam parameter or absorption non-finite or out of range
};

// Exact, order-independent accumulation of doubles (deterministic sums with
// atomics): a value x is scaled by 2^K, chosen per sum so that every partial
// sum stays below 2^92 in magnitude, and split into hi = floor(y / 2^32) and
// the integer part of y - hi 2^32 in [0, 2^32); both parts add as 64-bit
// integers, whose sum does not depend on the order.  Resolution 2^-K.
struct Fixed {
    unsigned long long hi, lo;
};
constexpr int kFixedBits = 92;

// Ray tracing: threads per workgroup (one ray each), the largest R_max (the
// face history of a ray is staged in LDS) and boxes per bounding group.
constexpr int kTraceThreads = 128;
constexpr int kTraceMaxRefl = 32;
constexpr int kTraceGroup = 8;

// Broadband synthesis: the largest transform (one row of double2 in LDS).
constexpr int kIrMaxFft = 4096;

}  // namespace gbs

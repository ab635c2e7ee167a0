// Transport sweeps, quadrature reduction and the source prologue (gfx950).
//
// 2D sweep (eq. (transport_sweep) with the upwind flux of eq. (upwind)):
//   One wavefront owns one (instance, quadrant, group of DG directions).  Its 64 lanes are 64
//   consecutive mesh rows of a band; lane j processes column i of band k at step
//   t = k*P + i + j, so the lanes form a diagonal wavefront that walks the whole mesh band after
//   band without a pipeline restart.  The y-trace of lane j reaches lane j+1 one step later
//   through a cross-lane shuffle, the last lane of a band hands its traces to lane 0 of the next
//   band through an LDS ring indexed by column, and the x-trace stays in registers.  Each lane
//   solves the DG cell system of DG directions per step and accumulates their contribution to
//   rho in FP64, so one partial density per (instance, quadrant group) leaves the kernel.
//
//   Every quadrant is swept in reflected coordinates (the sweep always runs towards +x, +y):
//   flipping the sign of the odd Legendre modes maps the upwind DG system of any quadrant onto
//   the (+,+) one.  In those coordinates the Q1 cell system with a = |vx|/hx, b = |vy|/hy is
//     K = a (A (x) I) + b (I (x) A) + sigma_t I,   A = [[1, s3], [-s3, 3]]   (s3 = sqrt 3)
//   (A from the volume and outflow-edge terms of eq. (DG) in the orthonormal basis), solved in
//   closed form by block elimination: with X = aA + (b+sigma)I, Y = aA + (3b+sigma)I and
//   A^2 = 4A - 6I, the Schur complement X Y + 3 b^2 I = uA + wI is again a polynomial in A.
#include <type_traits>

#include "rte_internal.h"

namespace rte {
namespace {

constexpr double kS3 = 1.7320508075688772935;

struct Sweep2DArgs {
    int nx, ny, B, nbands, P, n_dir, nparts;
    int wpb;         // wavefronts per band: direction groups summed in LDS
    int nbc;         // bands in flight per workgroup (each with its own wpb wavefronts)
    int P2;          // steps between a wavefront's consecutive bands: max(P, 64 nbc)
    int total;       // steps of the workgroup's pipeline
    int gq[4];       // workgroups (blocks of W direction groups) per quadrant
    int qstart[4];   // first entry of each quadrant in the sorted direction table
    int qpad[4];     // padded table length of each quadrant
    long long ncell;
    double ghost;            // sqrt(hx hy): coefficient of a unit constant on phi_0
    int zero_inflow;
    const DirEntry *dirs;
    const void *src;
    const double *inflow;
    double *partial;
    void *f_out;
    int ring_off;            // LDS offset (in doubles) of the y-trace rings
    const int *active;
    // material tables: with mat_ok set, the table kernel sweeps the instances with mat_ok[b] != 0
    // and the per-cell kernel the others
    const int *mat_ok;       // [B] or null
    const void *mcoef;       // [B][n_sorted][kMaxMat][8] T (mat_coef_kernel)
    int n_sorted;
    int mcoef_off;           // LDS offset (in doubles) of the workgroup's copy of its table rows
};

__device__ __forceinline__ float recip(float x);
__device__ __forceinline__ double recip(double x);

// Per-direction constants of the Q1 cell solve in reflected coordinates (a = |vx|/hx,
// b = |vy|/hy); with p = b + sigma and q = 3b + sigma the Schur-complement coefficients are
//   u = a (4a + p + q) = 4a(a + b) + 2a sigma,   w = p q + 3b^2 - 6a^2 = sigma (sigma + 4b) + 6(b^2 - a^2)
// so every cell-dependent quantity is one or two fused operations on sigma.
template <typename T>
struct DirConst {
    T al, be, ca, cb;       // a, b, s3 a, s3 b
    T k1, k2, k3, be4;      // 4a(a+b), 2a, 6(b^2-a^2), 4b
    T txc, twoal2;          // b + 2a, 2a^2
    T x00c, x11c;           // a + b, 3a + b
};

template <typename T>
__device__ __forceinline__ DirConst<T> dir_const(double a, double b) {
    DirConst<T> d;
    d.al = (T)a;
    d.be = (T)b;
    d.ca = (T)(kS3 * a);
    d.cb = (T)(kS3 * b);
    d.k1 = (T)(4.0 * a * (a + b));
    d.k2 = (T)(2.0 * a);
    d.k3 = (T)(6.0 * (b * b - a * a));
    d.be4 = (T)(4.0 * b);
    d.txc = (T)(b + 2.0 * a);
    d.twoal2 = (T)(2.0 * a * a);
    d.x00c = (T)(a + b);
    d.x11c = (T)(3.0 * a + b);
    return d;
}

// Q1 cell solve in reflected coordinates; unknown order k = a + 2b: (f00, f10, f01, f11).
// Block elimination with X = aA + pI, Y = aA + qI (A = [[1, s3], [-s3, 3]], A^2 = 4A - 6I):
//   (X Y + 3b^2 I) F1 = X R1 + s3 b R0  with  X Y + 3b^2 I = uA + wI,   F0 = X^{-1}(R0 - s3 b F1)
template <typename T>
__device__ __forceinline__ void q1_solve(const DirConst<T> &d, T sig, T r0, T r1, T r2, T r3,
                                         T &f0, T &f1, T &f2, T &f3) {
    const T c = T(kS3);
    const T u = d.k2 * sig + d.k1;
    const T w = sig * (sig + d.be4) + d.k3;
    const T tm = T(2) * u + w;
    const T detM = tm * tm + (u + u) * u;           // det(uA + wI) = (w+2u)^2 + 2u^2 > 0
    const T tx = sig + d.txc;
    const T detX = tx * tx + d.twoal2;              // det(X) = (p+2a)^2 + 2a^2 > 0
    const T inv = recip(detM * detX);
    const T iM = detX * inv;
    const T iX = detM * inv;
    const T x00 = sig + d.x00c;                     // a + p
    const T x11 = sig + d.x11c;                     // 3a + p
    const T g0 = x00 * r2 + (d.ca * r3 + d.cb * r0);
    const T g1 = x11 * r3 + (d.cb * r1 - d.ca * r2);
    const T cu = c * u;
    f2 = ((T(3) * u + w) * g0 - cu * g1) * iM;
    f3 = (cu * g0 + (u + w) * g1) * iM;
    const T h0 = r0 - d.cb * f2;
    const T h1 = r1 - d.cb * f3;
    f0 = (x11 * h0 - d.ca * h1) * iX;
    f1 = (d.ca * h0 + x00 * h1) * iX;
}

// wave-uniform value (all lanes hold the same number) moved to a scalar register
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ DirConst<T> uni(DirConst<T> d) {
    d.al = uni(d.al); d.be = uni(d.be); d.ca = uni(d.ca); d.cb = uni(d.cb);
    d.k1 = uni(d.k1); d.k2 = uni(d.k2); d.k3 = uni(d.k3); d.be4 = uni(d.be4);
    d.txc = uni(d.txc); d.twoal2 = uni(d.twoal2); d.x00c = uni(d.x00c); d.x11c = uni(d.x11c);
    return d;
}

// Cross-lane move "lane j receives lane j-1" as a DPP whole-wave shift (wave_shr:1).  Lane 0 has
// no source lane; with bound_ctrl off it keeps the instruction's old operand, which is the value
// lane 0 must receive (its inflow), so no select follows the shift.
__device__ __forceinline__ float shfl_up1(float lane0, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(lane0), __float_as_int(v),
                                                      0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double shfl_up1(double lane0, double v) {
    const long long b = __double_as_longlong(v), o = __double_as_longlong(lane0);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    const int olo = (int)(o & 0xffffffffll), ohi = (int)(o >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(olo, lo, 0x138, 0xf, 0xf, false);
    const int h2 = __builtin_amdgcn_update_dpp(ohi, hi, 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)h2 << 32) | (unsigned int)l2);
}

// reciprocal: hardware estimate refined by one Newton step (FP32), two steps (FP64)
__device__ __forceinline__ float recip(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return r * (2.0f - x * r);
}
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}

// Word 3 of a raw buffer resource on gfx9-family devices (32-bit data format; untyped loads and
// stores ignore the format beyond that), and a byte offset that is out of every range below 2 GiB.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kDropOffset = (int)0x80000000u;
constexpr int kStoreAux = 2;

// The 4 coefficients of one cell-direction through a raw buffer store (dropped by the hardware
// when the offset is outside the resource's range).
__device__ __forceinline__ void store_f4(__amdgpu_buffer_rsrc_t r, int off, const float (&v)[4]) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    v4i x;
    x.x = __float_as_int(v[0]); x.y = __float_as_int(v[1]);
    x.z = __float_as_int(v[2]); x.w = __float_as_int(v[3]);
    __builtin_amdgcn_raw_buffer_store_b128(x, r, off, 0, kStoreAux);
}
__device__ __forceinline__ void store_f4(__amdgpu_buffer_rsrc_t r, int off, const double (&v)[4]) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    v4i x, y;
    const long long a0 = __double_as_longlong(v[0]), a1 = __double_as_longlong(v[1]);
    const long long a2 = __double_as_longlong(v[2]), a3 = __double_as_longlong(v[3]);
    x.x = (int)a0; x.y = (int)(a0 >> 32); x.z = (int)a1; x.w = (int)(a1 >> 32);
    y.x = (int)a2; y.y = (int)(a2 >> 32); y.z = (int)a3; y.w = (int)(a3 >> 32);
    __builtin_amdgcn_raw_buffer_store_b128(x, r, off, 0, kStoreAux);
    __builtin_amdgcn_raw_buffer_store_b128(y, r, off + 16, 0, kStoreAux);
}

// One workgroup = W wavefronts per band = W consecutive direction groups of one (instance,
// quadrant), for nbc bands in flight.  The W wavefronts of a band walk the same pipeline in
// lockstep (one barrier per step), so at every step lane j of each is at the same cell; their
// FP64 partial densities are summed in LDS in a fixed order and one partial per (instance,
// quadrant block) is written.  With nbc > 1 the bands k, k+1, ... of the mesh run at once, band
// slot k mod nbc 64 steps behind the slot above it, which hands its last row's y-traces on
// through an LDS ring: the same cells, solves and sums in the same order as with one band in
// flight, over fewer dependent steps (a band no longer waits for the whole band above).
// MAT: the cell solve's coefficients that depend on sigma_t come from the instance's material
// table (the sweep input then carries the cell's material index in place of sigma_t).
template <typename T, int DG, bool WF, int NB, bool MAT>
__global__ void __launch_bounds__(256 * NB) sweep2d_kernel(Sweep2DArgs a) {
    extern __shared__ double smem_d[];
    const int lane = threadIdx.x & 63;
    const int W = (blockDim.x >> 6) / NB;                     // wavefronts per band
    const int wv = NB == 1 ? (int)(threadIdx.x >> 6) : (int)(threadIdx.x >> 6) % W;  // direction group
    const int kb = NB == 1 ? 0 : (int)(threadIdx.x >> 6) / W;                        // band slot
    const int item = blockIdx.x;                              // (instance, quadrant block)
    if (item >= a.B * a.nparts) return;                       // whole workgroup leaves
    const int b = item / a.nparts;
    const int gpart = item - b * a.nparts;
    if (a.active && a.active[b] == 0) return;
    if (a.mat_ok && (a.mat_ok[b] != 0) != MAT) return;    // the other kernel's instance
    int part = gpart, q = 0;
    while (q < 3 && part >= a.gq[q]) { part -= a.gq[q]; ++q; }
    const int g = part * W + wv;                              // direction group of this wave
    const int d0 = a.qstart[q] + g * DG;
    const int dend = a.qstart[q] + a.qpad[q];                 // end of this quadrant's table
    const bool rx = (q & 1) != 0, ry = (q & 2) != 0;
    // LDS: per band slot [2][W][64][4] doubles of partial densities (double buffered by step
    // parity), then per (band slot, direction group) a ring of y-traces, written by lane 63 and
    // read by lane 0 of the same direction group in the next band's slot
    double *red = smem_d + (size_t)kb * 2 * W * 64 * 4;
    const size_t ring_len = (size_t)a.nx * DG * 2;
    T *ring = reinterpret_cast<T *>(smem_d + a.ring_off) + ((size_t)kb * W + wv) * ring_len;
    const T *ring_in = NB == 1 ? ring
                               : reinterpret_cast<const T *>(smem_d + a.ring_off) +
                                     ((size_t)((kb + NB - 1) % NB) * W + wv) * ring_len;

    DirConst<T> dc[DG];
    T wt[DG];
    int orig[DG];
    const T c = T(kS3);
#pragma unroll
    for (int d = 0; d < DG; ++d) {
        DirEntry e;
        if (d0 + d < dend) e = a.dirs[d0 + d];
        else { e.alpha = 1.0; e.beta = 1.0; e.w = 0.0; e.orig = -1; e.pad = 0; }
        dc[d] = uni(dir_const<T>(e.alpha, e.beta));
        wt[d] = uni((T)e.w);
        orig[d] = __builtin_amdgcn_readfirstlane(e.orig);
    }
    const T gx = a.zero_inflow ? T(0) : (T)(a.inflow[4 * b + (rx ? 1 : 0)] * a.ghost);
    const T gy = a.zero_inflow ? T(0) : (T)(a.inflow[4 * b + (ry ? 3 : 2)] * a.ghost);
    const T sx = rx ? T(-1) : T(1), sy = ry ? T(-1) : T(1);
    const double dsx = rx ? -1.0 : 1.0, dsy = ry ? -1.0 : 1.0;

    // this quadrant's layout of the sweep inputs (see SweepLaunch)
    const bool la = quad_uses_a(q);
    const size_t nb4 = (size_t)a.B * a.ncell * 4;
    const T *base = reinterpret_cast<const T *>(a.src);
    const T *src = base + (la ? 0 : nb4) + (size_t)b * a.ncell * 4;
    const T *sig_t = base + 2 * nb4 + (la ? 0 : (size_t)a.B * a.ncell) + (size_t)b * a.ncell;
    double *part_out = a.partial ? a.partial + ((size_t)b * a.nparts + gpart) * a.ncell * 4 : nullptr;
    // angular flux [B][n_dir][cell][4], each direction's cells in band order (band_pos of the
    // reflected coordinates): at every step the lanes of a band are on consecutive positions
    // right after those of the previous step, so each store instruction writes one contiguous
    // run of 64 x 4 values and a wavefront's stores run through memory sequentially.  The
    // stores are raw buffer stores through one resource per direction whose range is that
    // direction's array: a lane without a value (outside the mesh, or a padding direction with
    // an empty range) gives an offset beyond the range and the hardware drops its store.  Every
    // lane issues every store, so the number of stores in flight is known at each step.
    __amdgpu_buffer_rsrc_t frs[WF ? DG : 1];
    if constexpr (WF) {
        T *fb = reinterpret_cast<T *>(a.f_out) + (size_t)b * a.n_dir * a.ncell * 4;
        const int bytes = (int)(a.ncell * 4 * (long long)sizeof(T));
#pragma unroll
        for (int d = 0; d < DG; ++d)
            frs[d] = __builtin_amdgcn_make_buffer_rsrc(
                fb + (size_t)(orig[d] >= 0 ? orig[d] : 0) * a.ncell * 4, 0,
                orig[d] >= 0 ? bytes : 0, kBufferWord3);
    }
    T tx0[DG], tx1[DG], ty0[DG], ty1[DG];
#pragma unroll
    for (int d = 0; d < DG; ++d) { tx0[d] = tx1[d] = ty0[d] = ty1[d] = T(0); }
    // the material table rows of the workgroup's W x DG directions, copied into LDS once (a
    // direction past the quadrant's padded table gets zeros: its values are never used)
    const Vec4<T> *mt = nullptr;
    if constexpr (MAT) {
        Vec4<T> *mtw = reinterpret_cast<Vec4<T> *>(smem_d + a.mcoef_off);
        const Vec4<T> *gm = reinterpret_cast<const Vec4<T> *>(a.mcoef) +
                            (size_t)b * a.n_sorted * kMaxMat * 2;
        const int first = a.qstart[q] + part * W * DG;
        for (int e = threadIdx.x; e < W * DG * kMaxMat * 2; e += blockDim.x) {
            const int di = first + e / (kMaxMat * 2);
            Vec4<T> v;
            v.x = v.y = v.z = v.w = T(0);
            if (di < dend) v = gm[(size_t)first * kMaxMat * 2 + e];
            mtw[e] = v;
        }
        __syncthreads();
        mt = mtw + (size_t)wv * DG * kMaxMat * 2;
    }

    // lane position in the pipeline: band k, column i (k P + i = t - lane), tracked
    // incrementally so the loop carries no division
    const int P2 = NB == 1 ? a.P : a.P2, nx = a.nx, ny = a.ny, nb = a.nbands;
    // position of the lane's cell in this quadrant's diagonal layout (inputs, partials)
    auto locate = [&](int kk, int ii, bool &ok) -> int {
        const int jr = kk * 64 + lane;
        ok = ii >= 0 && kk < nb && ii < nx && jr < ny;
        const int ip = rx ? nx - 1 - ii : ii;
        const int jp = ry ? ny - 1 - jr : jr;
        return ok ? (la ? pos_a(nx, ny, ip, jp) : pos_b(nx, ny, ip, jp)) : 0;
    };
    // cell data of one pipeline step: position (band k, column i) and the prefetched inputs
    struct CellIn {
        int k, i, pos;
        bool ok;
        Vec4<T> sv;
        T sg;
    };
    // Every lane loads (position 0 when outside the domain; such values are never used): a load
    // under a branch leaves the compiler unsure whether it was issued, and it then waits for it
    // at once instead of at the step that uses it.
    auto load_cell = [&](CellIn &c) {
        c.pos = locate(c.k, c.i, c.ok);
        c.sv = *reinterpret_cast<const Vec4<T> *>(src + (size_t)c.pos * 4);
        c.sg = sig_t[c.pos];
    };
    int rw = 0;     // the wavefront that sums this step's partial densities (step mod W)
    // One step: the lane's cell `cur` is solved while `nxt` is prefetched.  The loop below runs
    // steps in pairs with the two records swapping roles, so the prefetched data is consumed where
    // it was loaded (no register copy at the loop edge that would make the load land in its own
    // step).
    auto step = [&](int t, const CellIn &cur, CellIn &nxt) __attribute__((always_inline)) {
        // lane 0 takes its y-inflow from the boundary (first band) or from the ring.  Its position
        // is wave-uniform, so the branch is scalar and the ring read is one LDS broadcast; the
        // value enters the shift below as lane 0's operand.
        T r0v[DG], r1v[DG];
        {
            const int i0 = __builtin_amdgcn_readfirstlane(cur.i);
            const int k0 = __builtin_amdgcn_readfirstlane(cur.k);
            if (k0 == 0 || i0 < 0 || i0 >= nx || k0 >= nb) {
#pragma unroll
                for (int d = 0; d < DG; ++d) { r0v[d] = gy; r1v[d] = T(0); }
            } else {
#pragma unroll
                for (int d = 0; d < DG; ++d) {
                    r0v[d] = ring_in[(i0 * DG + d) * 2];
                    r1v[d] = ring_in[(i0 * DG + d) * 2 + 1];
                }
            }
        }
        T yi0[DG], yi1[DG];
#pragma unroll
        for (int d = 0; d < DG; ++d) {               // all lanes take part in the shift
            yi0[d] = shfl_up1(r0v[d], ty0[d]);
            yi1[d] = shfl_up1(r1v[d], ty1[d]);
        }
        // next position and prefetch of its cell data (overlaps this step's arithmetic)
        nxt.k = cur.k;
        nxt.i = cur.i + 1;
        if (nxt.i == P2) { nxt.i = 0; nxt.k += NB; }
        load_cell(nxt);
        // the lane's DG directions are summed in T, the groups and quadrants in FP64.
        // With f, every lane runs the arithmetic, also a lane outside the mesh: its values never
        // reach a lane inside it (at the next step lane j + 1 sits at lane j's column, so both
        // are outside together, and a lane entering a row resets its traces), its partial sums
        // are ignored and its f stores are dropped.  With no branch around them the stores are
        // issued as soon as a direction's values exist, and the compiler counts them exactly.
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
        if (WF || cur.ok) {
            if (cur.i == 0) {
#pragma unroll
                for (int d = 0; d < DG; ++d) { tx0[d] = gx; tx1[d] = T(0); }
            }
            const int off = (WF && cur.ok)
                                ? band_pos(nx, ny, cur.i, cur.k * 64 + lane) * (int)(4 * sizeof(T))
                                : kDropOffset;
            const T s0 = cur.sv.x, s1 = sx * cur.sv.y, s2 = sy * cur.sv.z, s3 = sx * sy * cur.sv.w;
            const T sig = cur.sg;
            T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
#pragma unroll
            for (int d = 0; d < DG; ++d) {
                const T r0 = s0 + dc[d].al * tx0[d] + dc[d].be * yi0[d];
                const T r1 = s1 - dc[d].ca * tx0[d] + dc[d].be * yi1[d];
                const T r2 = s2 + dc[d].al * tx1[d] - dc[d].cb * yi0[d];
                const T r3 = s3 - dc[d].ca * tx1[d] - dc[d].cb * yi1[d];
                T f0, f1, f2, f3;
                if constexpr (MAT) {
                    // (x00, x11, (3u + w)/detM, s3 u/detM), ((u + w)/detM, x11/detX, x00/detX,
                    // s3 a/detX) of the cell's material: q1_solve with its divisions folded in
                    const int m = (int)sig & (kMaxMat - 1);
                    const Vec4<T> c0 = mt[(d * kMaxMat + m) * 2];
                    const Vec4<T> c1 = mt[(d * kMaxMat + m) * 2 + 1];
                    const T g0 = c0.x * r2 + (dc[d].ca * r3 + dc[d].cb * r0);
                    const T g1 = c0.y * r3 + (dc[d].cb * r1 - dc[d].ca * r2);
                    f2 = c0.z * g0 - c0.w * g1;
                    f3 = c0.w * g0 + c1.x * g1;
                    const T h0 = r0 - dc[d].cb * f2;
                    const T h1 = r1 - dc[d].cb * f3;
                    f0 = c1.y * h0 - c1.w * h1;
                    f1 = c1.w * h0 + c1.z * h1;
                } else {
                    q1_solve<T>(dc[d], sig, r0, r1, r2, r3, f0, f1, f2, f3);
                }
                tx0[d] = f0 + c * f1;
                tx1[d] = f2 + c * f3;
                ty0[d] = f0 + c * f2;
                ty1[d] = f1 + c * f3;
                a0 += wt[d] * f0;
                a1 += wt[d] * f1;
                a2 += wt[d] * f2;
                a3 += wt[d] * f3;
                if constexpr (WF) {
                    const T fo[4] = {f0, sx * f1, sy * f2, sx * sy * f3};
                    store_f4(frs[d], off, fo);
                }
            }
            if (cur.ok && lane == 63) {
#pragma unroll
                for (int d = 0; d < DG; ++d) {
                    ring[(cur.i * DG + d) * 2] = ty0[d];
                    ring[(cur.i * DG + d) * 2 + 1] = ty1[d];
                }
            }
            acc0 = (double)a0;
            acc1 = (double)a1;
            acc2 = (double)a2;
            acc3 = (double)a3;
        }
        if (part_out) {
            // partial densities of this cell from every wavefront into LDS (double buffered by
            // step parity, so one barrier per step suffices), then their fixed-order sum by
            // wavefront 0
            double *slot = red + (size_t)(t & 1) * W * 64 * 4;
            {
                double4 v;
                v.x = acc0; v.y = acc1; v.z = acc2; v.w = acc3;
                *reinterpret_cast<double4 *>(slot + ((size_t)wv * 64 + lane) * 4) = v;
            }
            __syncthreads();
            // the summing wavefront rotates with the step, so the W wavefronts (on different
            // SIMDs) share that work evenly; the order of the sum is the same for all
            if (wv == rw && cur.ok) {
                double4 sum = *reinterpret_cast<const double4 *>(slot + (size_t)lane * 4);
                for (int w2 = 1; w2 < W; ++w2) {
                    const double4 o = *reinterpret_cast<const double4 *>(slot + ((size_t)w2 * 64 + lane) * 4);
                    sum.x += o.x; sum.y += o.y; sum.z += o.z; sum.w += o.w;
                }
                sum.y *= dsx; sum.z *= dsy; sum.w *= dsx * dsy;
                *reinterpret_cast<double4 *>(part_out + (size_t)cur.pos * 4) = sum;
            }
        }
        // The ring passes values between lanes of one wavefront (written by lane 63, read by
        // lane 0 at a later step, the very next one when the pipeline stride P is 64).  Within
        // one lane's program the write and the read never both run, so the compiler could move a
        // step's read above the previous step's write.  The barrier of the partial sums keeps
        // them in order; without partial sums this compiler-only barrier does (no instruction:
        // the LDS executes one wavefront's accesses in program order).
        if constexpr (WF) asm volatile("" ::: "memory");
        // with several bands in flight the ring links different wavefronts: a barrier per step
        // (the partial sums above already hold one)
        if constexpr (NB > 1) {
            if (!part_out) __syncthreads();
        }
        rw = rw + 1 == W ? 0 : rw + 1;
    };
    CellIn A, B;
    A.k = kb;                                  // band slot kb starts 64 kb steps after slot 0
    A.i = -lane - 64 * kb;
    load_cell(A);
    const int total = NB == 1 ? nb * a.P + 63 : a.total;
    int t = 0;
    for (; t + 1 < total; t += 2) {
        step(t, A, B);
        step(t + 1, B, A);
    }
    if (t < total) step(t, A, B);
}

// ------------------------------------------------------------------------------------- 1D
template <typename T>
__global__ void __launch_bounds__(256) sweep1d_kernel(int nc, int n_dir, int B, const double *mu,
                                                      const double *widths, const double *sigma_t,
                                                      const T *src, const double *inflow,
                                                      int zero_inflow, T *f_out,
                                                      const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * n_dir) return;
    const int b = (int)(t / n_dir), j = (int)(t - (long long)b * n_dir);
    if (active && active[b] == 0) return;
    const double m = mu[j];
    const bool rev = m < 0.0;
    const T am = (T)fabs(m);
    const T c = T(kS3);
    T edge = zero_inflow ? T(0) : (T)inflow[4 * b + (rev ? 1 : 0)];   // physical inflow value
    const T *s = src + (size_t)b * nc * 2;
    T *f = f_out + (size_t)b * nc * n_dir * 2 + (size_t)j * 2;    // [B][cell][n_dir][2]
    for (int st = 0; st < nc; ++st) {
        const int cc = rev ? nc - 1 - st : st;
        const T h = (T)widths[cc];
        const T sq = sqrt(h);
        const T aa = am / h;
        const T sig = (T)sigma_t[(size_t)b * nc + cc];
        const T e = am * edge / sq;               // |mu| f_edge phi_0(inflow edge)
        const T r0 = s[2 * cc] + e;
        const T r1 = (rev ? -s[2 * cc + 1] : s[2 * cc + 1]) - c * e;
        const T tt = sig + T(2) * aa;
        const T det = tt * tt + T(2) * aa * aa;
        const T f0 = ((T(3) * aa + sig) * r0 - c * aa * r1) / det;
        const T f1 = (c * aa * r0 + (aa + sig) * r1) / det;
        f[(size_t)cc * n_dir * 2] = f0;
        f[(size_t)cc * n_dir * 2 + 1] = rev ? -f1 : f1;
        edge = (f0 + c * f1) / sq;                 // outflow trace value
    }
}

// ------------------------------------------------------------------ source, reductions
// mat / mat_ok (2D, nullable): an instance with mat_ok[b] != 0 gets each cell's material index in
// place of its sigma_t (the table kernel of the sweep reads it)
template <typename T>
__global__ void source_kernel(int dim, long long ncell, int K, int B, int nx, int ny,
                              const double *rho, const double *sigma_t, const double *sigma_s,
                              const double *G, const double *cellw, double ghost, T *src,
                              const int *active, const int *mat, const int *mat_ok) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * ncell) return;
    const int b = (int)(t / ncell);
    if (active && active[b] == 0) return;
    const long long cell = t - (long long)b * ncell;
    const double ss = sigma_s[t];
    const double g0 = G ? G[t] * (cellw ? sqrt(cellw[cell]) : ghost) : 0.0;   // G null: no source
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k) v[k] = ss * rho[t * K + k] + (k == 0 ? g0 : 0.0);
    const double st = mat && mat_ok[b] ? (double)mat[t] : sigma_t[t];
    write_sweep_input<T>(dim, ncell, B, b, nx, ny, cell, v, st, src);
}

// ------------------------------------------------------------------ materials
// The distinct sigma_t values of each selected instance, ascending (at most kMaxMat), in two
// levels so that one large instance spreads over many workgroups.  Level one: every chunk of
// kMatChunk cells lists its smallest kMaxMat + 1 distinct values (INFINITY past its last), round
// r finding the smallest value above round r - 1's by a block-wide minimum.  Level two merges the
// chunk lists the same way.  An instance with at most kMaxMat values has every chunk list
// complete; one with more has more than kMaxMat in some chunk or in the union, and the merge
// sees kMaxMat + 1.
constexpr int kMatChunk = 4096;
constexpr int kMatList = kMaxMat + 1;

__device__ __forceinline__ double block_min256(double v, double *wmin) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = v;
    __syncthreads();
    v = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
    __syncthreads();
    return v;
}

// grid (chunks, B), 256 threads: cvals [B][chunks][kMatList]
__global__ void __launch_bounds__(256) mat_scan_kernel(long long ncell, const double *sigma_t,
                                                       const int *mask, double *cvals) {
    __shared__ double wmin[4];
    const int b = blockIdx.y;
    if (mask && mask[b] == 0) return;
    const long long c0 = (long long)blockIdx.x * kMatChunk;
    const long long c1 = c0 + kMatChunk < ncell ? c0 + kMatChunk : ncell;
    const double *sb = sigma_t + (size_t)b * ncell;
    double *out = cvals + ((size_t)b * gridDim.x + blockIdx.x) * kMatList;
    double last = -INFINITY;
    for (int r = 0; r < kMatList; ++r) {
        double mn = INFINITY;
        for (long long c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
            const double v = sb[c];
            if (v > last && v < mn) mn = v;
        }
        mn = block_min256(mn, wmin);
        if (threadIdx.x == 0) out[r] = mn;
        last = mn;
    }
}

// grid B, 256 threads: vals [B][kMaxMat] ascending, nmat [B], mat_ok [B] (0: more than kMaxMat)
__global__ void __launch_bounds__(256) mat_merge_kernel(int chunks, const double *cvals,
                                                        const int *mask, double *vals, int *nmat,
                                                        int *mat_ok) {
    __shared__ double wmin[4];
    const int b = blockIdx.x;
    if (mask && mask[b] == 0) return;
    const double *cb = cvals + (size_t)b * chunks * kMatList;
    const int n_all = chunks * kMatList;
    double last = -INFINITY;
    int n = 0;
    bool over = false;
    for (int r = 0; r < kMatList; ++r) {
        double mn = INFINITY;
        for (int k = threadIdx.x; k < n_all; k += blockDim.x) {
            const double v = cb[k];
            if (v > last && v < mn) mn = v;
        }
        mn = block_min256(mn, wmin);
        if (!(mn < INFINITY)) break;
        if (n == kMaxMat) {
            over = true;
            break;
        }
        if (threadIdx.x == 0) vals[(size_t)b * kMaxMat + n] = mn;
        ++n;
        last = mn;
    }
    if (threadIdx.x == 0) {
        nmat[b] = n;
        mat_ok[b] = over ? 0 : 1;
    }
}

// each cell's index in its instance's value list; a cell whose value is not there (a NaN)
// sends the instance to the per-cell kernel
__global__ void mat_map_kernel(long long ncell, const double *sigma_t, const int *mask,
                               const double *vals, const int *nmat, int *mat, int *mat_ok) {
    const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if ((mask && mask[b] == 0) || cell >= ncell) return;
    const size_t t = (size_t)b * ncell + cell;
    const double v = sigma_t[t];
    const int n = nmat[b];
    int m = -1;
    for (int j = 0; j < n; ++j)
        if (vals[(size_t)b * kMaxMat + j] == v) m = j;
    if (m < 0) {
        mat_ok[b] = 0;
        m = 0;
    }
    mat[t] = m;
}

// The sigma_t-dependent coefficients of the Q1 cell solve (q1_solve's u, w, det M, det X and
// the diagonal entries) for every (instance, sorted direction, material), in FP64 and stored in
// T: x00, x11, (3u + w)/det M, s3 u/det M, (u + w)/det M, x11/det X, x00/det X, s3 a/det X.
template <typename T>
__global__ void mat_coef_kernel(int B, int n_sorted, const DirEntry *dirs, const int *mask,
                                const double *vals, const int *nmat, T *coef) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)B * n_sorted * kMaxMat) return;
    const int m = (int)(t % kMaxMat);
    const long long bd = t / kMaxMat;
    const int di = (int)(bd % n_sorted), b = (int)(bd / n_sorted);
    if (mask && mask[b] == 0) return;
    T *o = coef + (size_t)t * 8;
    if (m >= nmat[b]) {
        for (int k = 0; k < 8; ++k) o[k] = T(0);
        return;
    }
    const double al = dirs[di].alpha, be = dirs[di].beta, sg = vals[(size_t)b * kMaxMat + m];
    const double u = 2.0 * al * sg + 4.0 * al * (al + be);
    const double w = sg * (sg + 4.0 * be) + 6.0 * (be * be - al * al);
    const double tm = 2.0 * u + w;
    const double detM = tm * tm + 2.0 * u * u;
    const double tx = sg + be + 2.0 * al;
    const double detX = tx * tx + 2.0 * al * al;
    const double iM = 1.0 / detM, iX = 1.0 / detX;
    const double x00 = sg + al + be, x11 = sg + 3.0 * al + be;
    o[0] = (T)x00;
    o[1] = (T)x11;
    o[2] = (T)((3.0 * u + w) * iM);
    o[3] = (T)(kS3 * u * iM);
    o[4] = (T)((u + w) * iM);
    o[5] = (T)(x11 * iX);
    o[6] = (T)(x00 * iX);
    o[7] = (T)(kS3 * al * iX);
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void max_update(unsigned long long *dst, double v) {
    // non-negative doubles order like their bit patterns; max is exact, hence deterministic
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

// rho* of one cell (4 dofs) = sum of the partial densities of every quadrant block, each read
// from its quadrant's diagonal layout, in fixed order.  Workgroups cover 16 x 16 cell tiles: a
// tile's cells on one diagonal sit on consecutive positions of either layout, so the reads of a
// workgroup fill whole cache lines.
struct ReduceArgs {
    long long ncell;
    int B, nx, ny, nparts;
    int gq[4];
};

__global__ void __launch_bounds__(256) reduce_parts_kernel(ReduceArgs a, int tiles_x,
                                                           const double *partial,
                                                           double *rho_star,
                                                           const double *rho_prev,
                                                           unsigned long long *maxd,
                                                           unsigned long long *maxr,
                                                           const int *active) {
    const int b = (int)(blockIdx.y);
    const int x = (int)(blockIdx.x % tiles_x) * 16 + (int)(threadIdx.x & 15);
    const int y = (int)(blockIdx.x / tiles_x) * 16 + (int)(threadIdx.x >> 4);
    const long long cell = (long long)y * a.nx + x;
    double d = 0.0, m = 0.0;
    const bool live = x < a.nx && y < a.ny && (!active || active[b] != 0);
    if (live) {
        const size_t pa = (size_t)pos_a(a.nx, a.ny, x, y);
        const size_t pb = (size_t)pos_b(a.nx, a.ny, x, y);
        const double *base = partial + (size_t)b * a.nparts * a.ncell * 4;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int part = 0;
        for (int q = 0; q < 4; ++q) {
            const size_t pos = quad_uses_a(q) ? pa : pb;
            for (int g = 0; g < a.gq[q]; ++g, ++part) {
                const double4 v = *reinterpret_cast<const double4 *>(base + ((size_t)part * a.ncell + pos) * 4);
                s0 += v.x; s1 += v.y; s2 += v.z; s3 += v.w;
            }
        }
        double4 o;
        o.x = s0; o.y = s1; o.z = s2; o.w = s3;
        const size_t gi = ((size_t)b * a.ncell + cell) * 4;
        *reinterpret_cast<double4 *>(rho_star + gi) = o;
        m = fmax(fmax(fabs(s0), fabs(s1)), fmax(fabs(s2), fabs(s3)));
        if (rho_prev)
            d = fmax(fmax(fabs(s0 - rho_prev[gi]), fabs(s1 - rho_prev[gi + 1])),
                     fmax(fabs(s2 - rho_prev[gi + 2]), fabs(s3 - rho_prev[gi + 3])));
    }
    if (maxd) max_update(maxd + b, d);
    if (maxr) max_update(maxr + b, m);
}

// 2D quadrature reduction of an angular flux in the sweep's layout [B][n_dir][cell][4] for the
// directions of one quadrant q.  A thread owns one stored position (band order of q's reflected
// coordinates), so for every direction a wavefront reads one contiguous run; the sums go to the
// natural cell (written by the pass of quadrant 0, added by the others).
template <typename T>
__global__ void scalar_flux2d_kernel(int nx, int ny, long long ncell, int n_dir, const double *vxy,
                                     const double *w, const T *f, double *rho, int q) {
    const long long pos = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)blockIdx.y;
    if (pos >= ncell) return;
    const long long cell = unreflect(nx, ny, band_cell(nx, ny, (int)pos), q);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 0; j < n_dir; ++j) {
        const int qj = (vxy[j] < 0.0 ? 1 : 0) | (vxy[n_dir + j] < 0.0 ? 2 : 0);
        if (qj != q) continue;
        const Vec4<T> v = *reinterpret_cast<const Vec4<T> *>(f + (((size_t)b * n_dir + j) * ncell + pos) * 4);
        const double wj = w[j];
        s0 += wj * (double)v.x; s1 += wj * (double)v.y; s2 += wj * (double)v.z; s3 += wj * (double)v.w;
    }
    double4 *o = reinterpret_cast<double4 *>(rho + ((size_t)b * ncell + cell) * 4);
    double4 r;
    if (q == 0) { r.x = s0; r.y = s1; r.z = s2; r.w = s3; }
    else {
        r = *o;
        r.x += s0; r.y += s1; r.z += s2; r.w += s3;
    }
    *o = r;
}

// 1D quadrature reduction (the slab sweep's f layout [B][cell][n_dir][K]), with the per-instance
// maxima of |rho| and of the change against rho_prev
template <typename T>
__global__ void scalar_flux_kernel(long long ndof, int K, int B, int n_dir, const double *w, const T *f,
                                   double *rho, const double *rho_prev, unsigned long long *maxd,
                                   unsigned long long *maxr, const int *active) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = (int)(blockIdx.y);
    double d = 0.0, m = 0.0;
    const bool live = t < ndof && (!active || active[b] != 0);
    if (live) {
        const long long c = t / K, k = t - c * K;              // f: [B][cell][n_dir][K]
        const T *fb = f + ((size_t)b * (ndof / K) + c) * n_dir * K + k;
        double s = 0.0;
        for (int j = 0; j < n_dir; ++j) s += w[j] * (double)fb[(size_t)j * K];
        rho[(size_t)b * ndof + t] = s;
        m = fabs(s);
        if (rho_prev) d = fabs(s - rho_prev[(size_t)b * ndof + t]);
    }
    if (maxd) max_update(maxd + b, d);
    if (maxr) max_update(maxr + b, m);
}

__global__ void check_kernel(long long n, const double *st, const double *ss, const double *g,
                             int *bad) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double a = st[t], s = ss[t], G = g[t];
    const bool ok = isfinite(a) && isfinite(s) && isfinite(G) && s >= 0.0 && a >= s;
    if (!ok) atomicOr(bad, 1);
}

template <typename T, int DG>
hipError_t sweep2d_launch_t(const SweepLaunch &L, hipStream_t s) {
    const rte_problem *p = L.p;
    Sweep2DArgs a;
    a.nx = p->nx;
    a.ny = p->ny;
    a.B = p->B;
    a.nbands = (p->ny + 63) / 64;
    a.P = p->nx > 64 ? p->nx : 64;
    a.n_dir = p->n_dir;
    const int W = sweep_waves(p);
    a.nparts = 0;
    for (int q = 0; q < 4; ++q) {
        const int groups = (p->quad.count[q] + DG - 1) / DG;
        a.gq[q] = (groups + W - 1) / W;
        a.qstart[q] = p->quad.start[q];
        a.qpad[q] = (p->quad.count[q] + kQuadPad - 1) / kQuadPad * kQuadPad;
        a.nparts += a.gq[q];
    }
    a.ncell = p->ncell;
    a.ghost = sqrt(p->hx * p->hy);
    a.zero_inflow = L.zero_inflow;
    a.dirs = p->d_dirs;
    a.src = L.src;
    a.inflow = p->inflow;
    a.partial = L.partial;
    a.f_out = L.f_out;
    a.active = L.active;
    a.mat_ok = L.mat_ok;
    a.mcoef = L.mat_coef;
    a.n_sorted = p->n_sorted;
    const unsigned grid = (unsigned)((long long)a.B * a.nparts);
    // bands in flight: the launch's choice, else the handle's, within what the mesh, the
    // workgroup size and the LDS budget allow
    const int NB = bands_in_flight(p, L.bands > 0 ? L.bands : sweep_bands(p), L.partial != nullptr,
                                   sizeof(T));
    a.wpb = W;
    a.nbc = NB;
    a.P2 = a.P > 64 * NB ? a.P : 64 * NB;
    // the last band (nbands - 1) sits in round (nbands - 1) / NB, slot (nbands - 1) % NB
    a.total = (a.nbands - 1) / NB * a.P2 + 64 * ((a.nbands - 1) % NB) + a.P + 63;
    // per band slot: partial-sum buffers (only when partial densities are formed); then the
    // y-trace rings of every (band slot, direction group)
    const size_t red = L.partial ? (size_t)NB * 2 * W * 64 * 4 * sizeof(double) : 0;
    const size_t lds = red + (size_t)NB * W * p->nx * DG * 2 * sizeof(T);
    a.ring_off = (int)(red / sizeof(double));
    // the table kernel's rows of its W x DG directions follow the rings
    a.mcoef_off = (int)(lds / sizeof(double));
    const size_t lds_mat = lds + (size_t)W * DG * kMaxMat * 2 * sizeof(Vec4<T>);
    const dim3 blk(64 * W * NB);
    auto go = [&](auto mat) {
        constexpr bool M = decltype(mat)::value;
        const size_t sh = M ? lds_mat : lds;
        switch (NB) {
            case 1:
                if (L.f_out) hipLaunchKernelGGL((sweep2d_kernel<T, DG, true, 1, M>), dim3(grid), blk, sh, s, a);
                else hipLaunchKernelGGL((sweep2d_kernel<T, DG, false, 1, M>), dim3(grid), blk, sh, s, a);
                break;
            case 2:
                if (L.f_out) hipLaunchKernelGGL((sweep2d_kernel<T, DG, true, 2, M>), dim3(grid), blk, sh, s, a);
                else hipLaunchKernelGGL((sweep2d_kernel<T, DG, false, 2, M>), dim3(grid), blk, sh, s, a);
                break;
            default:
                if (L.f_out) hipLaunchKernelGGL((sweep2d_kernel<T, DG, true, 4, M>), dim3(grid), blk, sh, s, a);
                else hipLaunchKernelGGL((sweep2d_kernel<T, DG, false, 4, M>), dim3(grid), blk, sh, s, a);
                break;
        }
    };
    // with tables: the table kernel for the instances that have one, then the per-cell kernel
    // for the others (its workgroups of table instances leave at once)
    if (L.mat_ok) go(std::true_type{});
    go(std::false_type{});
    return hipGetLastError();
}

// the dynamic LDS limit of every 2D sweep kernel (the table kernels go past 64 KiB)
template <typename T, int DG>
void sweep_lds_limit_t(int bytes) {
    auto set = [&](const void *f) {
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    };
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 1, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 1, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 2, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 2, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 4, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 4, false>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 1, true>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 1, true>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 2, true>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 2, true>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, false, 4, true>));
    set(reinterpret_cast<const void *>(&sweep2d_kernel<T, DG, true, 4, true>));
}

template <typename T>
hipError_t sweep2d_dispatch(const SweepLaunch &L, hipStream_t s) {
    switch (L.p->tune.dg) {
        case 1: return sweep2d_launch_t<T, 1>(L, s);
        case 2: return sweep2d_launch_t<T, 2>(L, s);
        case 4: return sweep2d_launch_t<T, 4>(L, s);
        case 8: return sweep2d_launch_t<T, 8>(L, s);
        default: return hipErrorInvalidValue;
    }
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_sweep2d(const SweepLaunch &a, hipStream_t s) {
    return a.fp32 ? sweep2d_dispatch<float>(a, s) : sweep2d_dispatch<double>(a, s);
}

void sweep_lds_limits(int bytes) {
    sweep_lds_limit_t<float, 1>(bytes);
    sweep_lds_limit_t<float, 2>(bytes);
    sweep_lds_limit_t<float, 4>(bytes);
    sweep_lds_limit_t<float, 8>(bytes);
    sweep_lds_limit_t<double, 1>(bytes);
    sweep_lds_limit_t<double, 2>(bytes);
    sweep_lds_limit_t<double, 4>(bytes);
    sweep_lds_limit_t<double, 8>(bytes);
    (void)hipGetLastError();
}

size_t sweep_mat_lds_bytes(const rte_problem *p, size_t elem) {
    return (size_t)sweep_waves(p) * p->tune.dg * kMaxMat * 2 * 4 * elem;
}

bool sweep_mat_fits(const rte_problem *p, size_t elem) {
    // the largest workgroup of a table kernel: partial sums, rings at the most bands in flight
    // the handle's schedule can run, and the table rows
    const int NB = bands_in_flight(p, 4, true, elem);
    return sweep_lds_bytes(p, NB, true, elem) + sweep_mat_lds_bytes(p, elem) <=
           (size_t)p->lds_per_cu;
}

int mat_chunks(const rte_problem *p) { return (int)((p->ncell + kMatChunk - 1) / kMatChunk); }

hipError_t launch_materials(const rte_problem *p, const int *mask, int *mat, int *mat_ok,
                            int *nmat, double *vals, double *cvals, void *coef, int fp32,
                            hipStream_t s) {
    const int chunks = mat_chunks(p);
    hipLaunchKernelGGL(mat_scan_kernel, dim3(chunks, p->B), dim3(256), 0, s, p->ncell,
                       p->sigma_t, mask, cvals);
    hipLaunchKernelGGL(mat_merge_kernel, dim3(p->B), dim3(256), 0, s, chunks, cvals, mask, vals,
                       nmat, mat_ok);
    hipLaunchKernelGGL(mat_map_kernel, dim3(blocks_for(p->ncell, 256), p->B), dim3(256), 0, s,
                       p->ncell, p->sigma_t, mask, vals, nmat, mat, mat_ok);
    const long long n = (long long)p->B * p->n_sorted * kMaxMat;
    if (fp32)
        hipLaunchKernelGGL(mat_coef_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->B,
                           p->n_sorted, p->d_dirs, mask, vals, nmat, (float *)coef);
    else
        hipLaunchKernelGGL(mat_coef_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->B,
                           p->n_sorted, p->d_dirs, mask, vals, nmat, (double *)coef);
    return hipGetLastError();
}

hipError_t launch_sweep1d(const rte_problem *p, const void *src, void *f_out, const int *active,
                          int zero_inflow, int fp32, hipStream_t s) {
    const long long n = (long long)p->B * p->n_dir;
    if (fp32)
        hipLaunchKernelGGL(sweep1d_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->nx,
                           p->n_dir, p->B, p->d_mu, p->d_widths, p->sigma_t,
                           (const float *)src, p->inflow, zero_inflow, (float *)f_out, active);
    else
        hipLaunchKernelGGL(sweep1d_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->nx,
                           p->n_dir, p->B, p->d_mu, p->d_widths, p->sigma_t,
                           (const double *)src, p->inflow, zero_inflow, (double *)f_out, active);
    return hipGetLastError();
}

hipError_t launch_source(const rte_problem *p, const double *rho, void *src, const int *active,
                         int fp32, hipStream_t s, bool with_G, const int *mat,
                         const int *mat_ok) {
    const long long n = (long long)p->B * p->ncell;
    const double ghost = sqrt(p->hx * p->hy);
    const double *cw = p->dim == 1 ? p->d_widths : nullptr;
    const double *G = with_G ? p->source : nullptr;
    if (fp32)
        hipLaunchKernelGGL(source_kernel<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, p->dim,
                           p->ncell, p->K, p->B, p->nx, p->ny, rho, p->sigma_t, p->sigma_s,
                           G, cw, ghost, (float *)src, active, mat, mat_ok);
    else
        hipLaunchKernelGGL(source_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                           p->dim, p->ncell, p->K, p->B, p->nx, p->ny, rho, p->sigma_t,
                           p->sigma_s, G, cw, ghost, (double *)src, active, mat, mat_ok);
    return hipGetLastError();
}

hipError_t launch_reduce_parts(const rte_problem *p, const double *partial, int nparts,
                               double *rho_star, const double *rho_prev, unsigned long long *maxd,
                               unsigned long long *maxr, const int *active, hipStream_t s) {
    ReduceArgs a;
    a.ncell = p->ncell;
    a.B = p->B;
    a.nx = p->nx;
    a.ny = p->ny;
    a.nparts = nparts;
    const int W = p->tune.wpb, DG = p->tune.dg;
    for (int q = 0; q < 4; ++q) a.gq[q] = ((p->quad.count[q] + DG - 1) / DG + W - 1) / W;
    const int tx = (p->nx + 15) / 16, ty = (p->ny + 15) / 16;
    dim3 grid((unsigned)(tx * ty), p->B);
    hipLaunchKernelGGL(reduce_parts_kernel, grid, dim3(256), 0, s, a, tx, partial, rho_star,
                       rho_prev, maxd, maxr, active);
    return hipGetLastError();
}

hipError_t launch_scalar_flux(const rte_problem *p, const void *f, double *rho, int fp32,
                              const double *rho_prev, unsigned long long *maxd,
                              unsigned long long *maxr, const int *active, hipStream_t s) {
    if (p->dim == 2) {
        // the quadrant-0 pass writes every cell (a quadrant without directions contributes
        // zero), the others add; no change maxima in 2D (the sweep forms rho* itself)
        if (rho_prev || maxd || maxr || active) return hipErrorInvalidValue;
        dim3 g2(blocks_for(p->ncell, 256), p->B);
        for (int q = 0; q < 4; ++q) {
            if (fp32)
                hipLaunchKernelGGL(scalar_flux2d_kernel<float>, g2, dim3(256), 0, s, p->nx, p->ny,
                                   p->ncell, p->n_dir, p->d_vxy, p->d_w, (const float *)f, rho, q);
            else
                hipLaunchKernelGGL(scalar_flux2d_kernel<double>, g2, dim3(256), 0, s, p->nx, p->ny,
                                   p->ncell, p->n_dir, p->d_vxy, p->d_w, (const double *)f, rho, q);
        }
        return hipGetLastError();
    }
    dim3 grid(blocks_for(p->ndof, 256), p->B);
    if (fp32)
        hipLaunchKernelGGL(scalar_flux_kernel<float>, grid, dim3(256), 0, s, p->ndof, p->K, p->B, p->n_dir,
                           p->d_w, (const float *)f, rho, rho_prev, maxd, maxr, active);
    else
        hipLaunchKernelGGL(scalar_flux_kernel<double>, grid, dim3(256), 0, s, p->ndof, p->K, p->B,
                           p->n_dir, p->d_w, (const double *)f, rho, rho_prev, maxd, maxr, active);
    return hipGetLastError();
}

hipError_t launch_check_materials(const rte_problem *p, int *bad, hipStream_t s) {
    const long long n = (long long)p->B * p->ncell;
    hipLaunchKernelGGL(check_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, p->sigma_t,
                       p->sigma_s, p->source, bad);
    return hipGetLastError();
}

}  // namespace rte

namespace rte {
int sweep_waves(const rte_problem *p) { return p->tune.wpb; }
int sweep_bands(const rte_problem *p) { return p->tune.bands > 0 ? p->tune.bands : 1; }

size_t sweep_lds_bytes(const rte_problem *p, int bands, bool partial, size_t elem) {
    const int W = p->tune.wpb, DG = p->tune.dg;
    const size_t red = partial ? (size_t)bands * 2 * W * 64 * 4 * sizeof(double) : 0;
    return red + (size_t)bands * W * p->nx * DG * 2 * elem;
}

int bands_in_flight(const rte_problem *p, int requested, bool partial, size_t elem) {
    // the kernel is compiled for 1, 2 or 4 bands in flight
    int nb = requested >= 4 ? 4 : requested >= 2 ? 2 : 1;
    const int nbands = (p->ny + 63) / 64;
    while (nb > 1 && (nb > nbands || sweep_lds_bytes(p, nb, partial, elem) > kSweepLdsBytes))
        nb /= 2;
    return nb;
}

int sweep_bands_used(const rte_problem *p, rte_precision prec) {
    return bands_in_flight(p, sweep_bands(p), true, prec == RTE_MIXED ? sizeof(float) : sizeof(double));
}
int sweep_nparts(const rte_problem *p) {
    const int W = p->tune.wpb, DG = p->tune.dg;
    int n = 0;
    for (int q = 0; q < 4; ++q) {
        const int groups = (p->quad.count[q] + DG - 1) / DG;
        n += (groups + W - 1) / W;
    }
    return n;
}
}  // namespace rte

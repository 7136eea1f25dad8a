// ms_step.hip — fused batched rigid-body step for CDNA4 (gfx950).
//
// One 64-lane wavefront per workgroup.  A workgroup takes tiles from a static work list; a tile
// packs 64 / G envs and G lanes serve each env.  For the whole launch an env's bodies, contact
// rows, friction patches, joints and colour schedule live in LDS: HBM is read once at the start
// (state, body parameters, joints, drive targets) and written once at the end (state, status),
// however many steps the launch runs.
//
// Step model (the paper relies on a GPU rigid-body solver tuned by position / velocity
// iteration counts, App. E Setup, with PD joint drives, App. B; its equations are not given):
//   S0 frozen step-start pose, world inverse inertia and velocities;
//   S1 exact AABBs (no contraction: identical candidate lists on any IEEE-754 binary32 target);
//   S2 all pairs of the env in canonical (a, b) order, ground plane last, with the static-static
//      and jointed parent-child filters;
//   S3 narrowphase in a frame centred on body A (sphere, capsule, box, plane), <= 4 points;
//   S4 normal rows per point, one friction patch per manifold (two tangents + twist);
//   S5 greedy colouring over joints then manifolds; the colour order fixes the Gauss-Seidel order;
//   S6 substeps: gravity, warm start, joint-only passes, coloured sweep, integration of the
//      offsets from the step-start pose;
//   S7 velocity sweeps and the restitution pass; S8 non-finite guard and write-back.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ms_dev.h"

using namespace msdev;

namespace {

// ----------------------------------------------------------------------------- small math
struct V3 { float x, y, z; };
struct Qt { float w, x, y, z; };

__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator-(V3 a) { return {-a.x, -a.y, -a.z}; }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ float len3(V3 a) { return sqrtf(dot3(a, a)); }
// c ? a : b on values (component selects; no address of either operand is taken).
__device__ __forceinline__ V3 vsel(bool c, V3 a, V3 b) { return {c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z}; }
__device__ __forceinline__ float comp(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
__device__ __forceinline__ void setc(V3& a, int i, float v) {
    if (i == 0) a.x = v; else if (i == 1) a.y = v; else a.z = v;
}

__device__ __forceinline__ Qt qmul(Qt a, Qt b) {
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ Qt qnorm(Qt a) {
    float inv = 1.0f / sqrtf(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    return {a.w * inv, a.x * inv, a.y * inv, a.z * inv};
}

// 3x3 rotation (row-major) of a unit quaternion.
struct M3 { float m[3][3]; };
__device__ __forceinline__ M3 rotm(Qt q) {
    float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    M3 r;
    r.m[0][0] = 1.0f - 2.0f * (yy + zz); r.m[0][1] = 2.0f * (xy - wz);        r.m[0][2] = 2.0f * (xz + wy);
    r.m[1][0] = 2.0f * (xy + wz);        r.m[1][1] = 1.0f - 2.0f * (xx + zz); r.m[1][2] = 2.0f * (yz - wx);
    r.m[2][0] = 2.0f * (xz - wy);        r.m[2][1] = 2.0f * (yz + wx);        r.m[2][2] = 1.0f - 2.0f * (xx + yy);
    return r;
}
__device__ __forceinline__ V3 mulv(const M3& a, V3 v) {
    return {a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z, a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z,
            a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z};
}
__device__ __forceinline__ V3 mulTv(const M3& a, V3 v) {
    return {a.m[0][0] * v.x + a.m[1][0] * v.y + a.m[2][0] * v.z, a.m[0][1] * v.x + a.m[1][1] * v.y + a.m[2][1] * v.z,
            a.m[0][2] * v.x + a.m[1][2] * v.y + a.m[2][2] * v.z};
}
// Column j; every element is read at a constant offset (a run-time j selects between values),
// so matrices stay in registers.
__device__ __forceinline__ V3 colm(const M3& a, int j) {
    V3 c0 = {a.m[0][0], a.m[1][0], a.m[2][0]}, c1 = {a.m[0][1], a.m[1][1], a.m[2][1]}, c2 = {a.m[0][2], a.m[1][2], a.m[2][2]};
    return j == 0 ? c0 : (j == 1 ? c1 : c2);
}

// Symmetric 3x3 stored as xx, yy, zz, xy, xz, yz.
struct S6 { float xx, yy, zz, xy, xz, yz; };
__device__ __forceinline__ V3 muls(const S6& s, V3 v) {
    return {s.xx * v.x + s.xy * v.y + s.xz * v.z, s.xy * v.x + s.yy * v.y + s.yz * v.z,
            s.xz * v.x + s.yz * v.y + s.zz * v.z};
}

// ----------------------------------------------------------------------------- LDS layout
// (Lay / make_lay live in ms_dev.h: one definition for the kernel and the host planner)
// Contact-row words (one record per point): rA 0..2, rB 3..5, n 6..8, mn 9, s0 10, vnpre 11, ln 12,
// bias of the current substep 13.
enum { R_RA = 0, R_RB = 3, R_N = 6, R_MN = 9, R_S0 = 10, R_VN = 11, R_LN = 12, R_BIAS = 13 };
// Manifold words (one record per manifold): header 0 (a | b << 8 as int), 1 (first | count << 16),
// rA 2..4, rB 5..7, nb 8..10, t1 11..13, mt1 14, mt2 15, mtw 16, mu 17, rt 18, lt1 19, lt2 20, ltw 21,
// restitution 22.
enum { M_AB = 0, M_FC = 1, M_RA = 2, M_RB = 5, M_NB = 8, M_T1 = 11, M_MT1 = 14, M_MT2 = 15, M_MTW = 16,
       M_MU = 17, M_RT = 18, M_LT1 = 19, M_LT2 = 20, M_LTW = 21, M_REST = 22 };
// Joint record in LDS (31 words): parent, child, aA 2..4, QA 5..8, aB 9..11, QB 12..15, kp 16,
// kd 17, target 18, accumulated impulses of the step: lp 19..21 (revolute point block; prismatic
// rows across the slide axis in 19..20), la 22..24 (revolute angular block in 22..23; prismatic
// rotation lock), ld 25 (drive), ll 26..27 (lower / upper limit); type | limited << 8 28 (int),
// lower 29, upper 30.
enum { J_PA = 0, J_CH = 1, J_AA = 2, J_QA = 5, J_AB = 9, J_QB = 12, J_KP = 16, J_KD = 17, J_TG = 18,
       J_LP = 19, J_LA = 22, J_LD = 25, J_LL = 26, J_TYP = 28, J_LO = 29, J_HI = 30, J_WORDS = 31 };
// Scalars.
enum { SC_NCAND = 0, SC_NPTS = 1, SC_NMAN = 2, SC_NCOL = 3, SC_STATUS = 4, SC_NSCHED = 5, SC_NJSCHED = 6,
       SC_NDYN = 7 };

struct EnvCtx {
    float* L;       // LDS base of the env
    Lay lay;
    const BatchDev* bd;
    int env, b0, j0;
    bool active;
};

__device__ __forceinline__ int* iptr(float* p) { return reinterpret_cast<int*>(p); }

// HBM accesses through address-space-1 (global) pointers: global loads and stores, which the
// compiler may reorder freely against LDS accesses.  Through generic pointers it must emit flat
// accesses and order every one of them against the LDS writes around it (a flat address could be
// LDS), which serialises the loads of a phase into one HBM round trip each.
#define MS_GPTR(T, p) ((__attribute__((address_space(1))) T*)(p))
__device__ __forceinline__ float gld(const float* p) { return *MS_GPTR(const float, p); }
__device__ __forceinline__ int gldi(const int* p) { return *MS_GPTR(const int, p); }
__device__ __forceinline__ float4 gld4(const float4* p) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = *MS_GPTR(const f4, p);
    return float4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void gst(float* p, float v) { *MS_GPTR(float, p) = v; }
__device__ __forceinline__ void gsti(int* p, int v) { *MS_GPTR(int, p) = v; }
// 64-bit add to HBM without a return value (no wait for the old value)
__device__ __forceinline__ void gadd64(long long* p, long long v) {
    __hip_atomic_fetch_add(MS_GPTR(long long, p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint16_t* hptr(float* p) { return reinterpret_cast<uint16_t*>(p); }

__device__ __forceinline__ V3 ld3(const float* L, int off, int n, int i) {
    return {L[off + i], L[off + n + i], L[off + 2 * n + i]};
}
__device__ __forceinline__ void st3(float* L, int off, int n, int i, V3 v) {
    L[off + i] = v.x; L[off + n + i] = v.y; L[off + 2 * n + i] = v.z;
}
__device__ __forceinline__ Qt ld4(const float* L, int off, int n, int i) {
    return {L[off + i], L[off + n + i], L[off + 2 * n + i], L[off + 3 * n + i]};
}
__device__ __forceinline__ void st4(float* L, int off, int n, int i, Qt q) {
    L[off + i] = q.w; L[off + n + i] = q.x; L[off + 2 * n + i] = q.y; L[off + 3 * n + i] = q.z;
}

// ----------------------------------------------------------------------------- wave helpers
// Every workgroup is exactly one wavefront (64 lanes).  LDS operations of one wavefront are
// performed in program order, so lanes that exchange data through LDS between phases need only
// a wavefront-scope fence, which keeps the compiler from moving memory operations across the
// phase boundary and costs no wait on the hardware.
__device__ __forceinline__ int opaque_lane(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
    return v;
}
__device__ __forceinline__ uint64_t group_bits(uint64_t ballot, int g, int G) {
    return G == 64 ? ballot : (ballot >> (g * G)) & ((uint64_t(1) << G) - 1);
}
__device__ __forceinline__ int prefix_in_group(uint64_t gb, int li) {
    return __popcll(gb & ((uint64_t(1) << li) - 1));
}
// Exclusive prefix sum over the lanes of a group (G a power of two <= 64) and the group total,
// for 0 <= v < 2^BITS, from one ballot per bit (no cross-lane data movement).
template <int BITS>
__device__ __forceinline__ int group_scan_small(int v, int li, int g, int G, int& total) {
    int pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t m = group_bits(__ballot((v >> b) & 1), g, G);
        pre += prefix_in_group(m, li) << b;
        tot += __popcll(m) << b;
    }
    total = tot;
    return pre;
}

// ----------------------------------------------------------------------------- body access
struct BodyRef {
    float invm;
    S6 Iw;
    bool dyn;
};
__device__ __forceinline__ bool is_dyn(const EnvCtx& c, int i) {
    return i >= 0 && !((iptr(c.L + c.lay.SH)[i] >> 8) & 1);
}
__device__ __forceinline__ float* body_rec(const EnvCtx& c, int i) { return c.L + c.lay.BODY + i * BODY_WORDS; }
__device__ __forceinline__ float* pose_rec(const EnvCtx& c, int i) { return c.L + c.lay.POSE + i * POSE_WORDS; }
__device__ __forceinline__ V3 ldp3(const EnvCtx& c, int i, int w) { const float* R = pose_rec(c, i) + w; return v3(R[0], R[1], R[2]); }
__device__ __forceinline__ Qt ldp4(const EnvCtx& c, int i, int w) { const float* R = pose_rec(c, i) + w; return Qt{R[0], R[1], R[2], R[3]}; }
__device__ __forceinline__ void stp3(const EnvCtx& c, int i, int w, V3 v) { float* R = pose_rec(c, i) + w; R[0] = v.x; R[1] = v.y; R[2] = v.z; }
__device__ __forceinline__ void stp4(const EnvCtx& c, int i, int w, Qt q) { float* R = pose_rec(c, i) + w; R[0] = q.w; R[1] = q.x; R[2] = q.y; R[3] = q.z; }
__device__ __forceinline__ S6 load_iw(const EnvCtx& c, int i) {
    const float* R = body_rec(c, i) + B_IW;
    return S6{R[0], R[1], R[2], R[3], R[4], R[5]};
}
__device__ __forceinline__ V3 ldv(const EnvCtx& c, int i) { const float* R = body_rec(c, i) + B_V; return v3(R[0], R[1], R[2]); }
__device__ __forceinline__ V3 ldw(const EnvCtx& c, int i) { const float* R = body_rec(c, i) + B_W; return v3(R[0], R[1], R[2]); }
__device__ __forceinline__ void stv(const EnvCtx& c, int i, V3 v) { float* R = body_rec(c, i) + B_V; R[0] = v.x; R[1] = v.y; R[2] = v.z; }
__device__ __forceinline__ void stw(const EnvCtx& c, int i, V3 v) { float* R = body_rec(c, i) + B_W; R[0] = v.x; R[1] = v.y; R[2] = v.z; }

// ----------------------------------------------------------------------------- narrowphase
// Every array below is indexed by compile-time constants only (loops are unrolled and run-time
// choices become selects), so the narrowphase lives in registers, not in scratch memory.
struct Pt { V3 p, n; float s; };
// Contact points of one pair: up to 8 slots; the pair's point list is the valid slots (mask)
// in slot order.  Each generator writes its k-th candidate point into slot k.
struct NOut {
    Pt pt[8];
    uint32_t mask;
    int decision;
};
struct Shp {
    int type;
    V3 c;
    M3 R;
    float d[3];
    __device__ V3 p0() const { return c - d[1] * colm(R, 2); }
    __device__ V3 p1() const { return c + d[1] * colm(R, 2); }
};
__device__ __forceinline__ float dim(const Shp& s, int i) { return i == 0 ? s.d[0] : (i == 1 ? s.d[1] : s.d[2]); }
__device__ __forceinline__ V3 axis(const Shp& s, int i) {
    return i == 0 ? colm(s.R, 0) : (i == 1 ? colm(s.R, 1) : colm(s.R, 2));
}
// c ? a : b, field by field (a value select keeps both shapes in registers).
__device__ __forceinline__ Shp pick(bool c, const Shp& a, const Shp& b) {
    Shp r;
    r.type = c ? a.type : b.type;
    r.c = v3(c ? a.c.x : b.c.x, c ? a.c.y : b.c.y, c ? a.c.z : b.c.z);
    r.d[0] = c ? a.d[0] : b.d[0]; r.d[1] = c ? a.d[1] : b.d[1]; r.d[2] = c ? a.d[2] : b.d[2];
    r.R.m[0][0] = c ? a.R.m[0][0] : b.R.m[0][0]; r.R.m[0][1] = c ? a.R.m[0][1] : b.R.m[0][1];
    r.R.m[0][2] = c ? a.R.m[0][2] : b.R.m[0][2]; r.R.m[1][0] = c ? a.R.m[1][0] : b.R.m[1][0];
    r.R.m[1][1] = c ? a.R.m[1][1] : b.R.m[1][1]; r.R.m[1][2] = c ? a.R.m[1][2] : b.R.m[1][2];
    r.R.m[2][0] = c ? a.R.m[2][0] : b.R.m[2][0]; r.R.m[2][1] = c ? a.R.m[2][1] : b.R.m[2][1];
    r.R.m[2][2] = c ? a.R.m[2][2] : b.R.m[2][2];
    return r;
}
__device__ __forceinline__ int n_points(const NOut& o) { return __popc(o.mask); }

template <int K>
__device__ __forceinline__ void emit(NOut& o, V3 pa, V3 pb, V3 n, float s, float delta) {
    static_assert(K >= 0 && K < 8, "slot");
    if (s < delta) {
        o.pt[K].p = 0.5f * (pa + pb);
        o.pt[K].n = n;
        o.pt[K].s = s;
        o.mask |= 1u << K;
    }
}

__device__ __forceinline__ float clamp01(float v) { return v < 0.0f ? 0.0f : (v > 1.0f ? 1.0f : v); }

// Segment-segment closest parameters (clamped-parameter method, Ericson RTCD 5.1.9).
__device__ __forceinline__ void seg_seg(V3 p1, V3 q1, V3 p2, V3 q2, float& s, float& t) {
    V3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    float a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
    const float eps = 1e-12f;
    if (a <= eps && e <= eps) { s = 0.0f; t = 0.0f; return; }
    if (a <= eps) { s = 0.0f; t = clamp01(f / e); return; }
    float c = dot3(d1, r);
    if (e <= eps) { t = 0.0f; s = clamp01(-c / a); return; }
    float b = dot3(d1, d2);
    float den = a * e - b * b;
    s = den != 0.0f ? clamp01((b * f - c * e) / den) : 0.0f;
    t = (b * s + f) / e;
    if (t < 0.0f) { t = 0.0f; s = clamp01(-c / a); }
    else if (t > 1.0f) { t = 1.0f; s = clamp01((b - c) / a); }
}
__device__ __forceinline__ float seg_point(V3 p0, V3 p1, V3 x) {
    V3 d = p1 - p0;
    float dd = dot3(d, d);
    if (dd <= 1e-12f) return 0.0f;
    return clamp01(dot3(x - p0, d) / dd);
}

template <int K>
__device__ __forceinline__ void np_sphere_sphere(NOut& o, V3 ca, float ra, V3 cb, float rb, float delta) {
    V3 d = cb - ca;
    float dist = len3(d);
    V3 n = dist < 1e-9f ? v3(0.0f, 0.0f, 1.0f) : (1.0f / dist) * d;
    emit<K>(o, ca + ra * n, cb - rb * n, n, dist - ra - rb, delta);
}

template <int K>
__device__ __forceinline__ void np_plane_sphere(NOut& o, V3 c, float r, float delta) {
    V3 n = v3(0.0f, 0.0f, 1.0f);
    emit<K>(o, v3(c.x, c.y, 0.0f), c - r * n, n, c.z - r, delta);
}

template <int K>
__device__ __forceinline__ void plane_box_corner(NOut& o, const Shp& b, float delta) {
    V3 l = v3((K & 1) ? b.d[0] : -b.d[0], (K & 2) ? b.d[1] : -b.d[1], (K & 4) ? b.d[2] : -b.d[2]);
    V3 c = b.c + mulv(b.R, l);
    emit<K>(o, v3(c.x, c.y, 0.0f), c, v3(0.0f, 0.0f, 1.0f), c.z, delta);
}
__device__ __forceinline__ void np_plane_box(NOut& o, const Shp& b, float delta) {
    plane_box_corner<0>(o, b, delta); plane_box_corner<1>(o, b, delta);
    plane_box_corner<2>(o, b, delta); plane_box_corner<3>(o, b, delta);
    plane_box_corner<4>(o, b, delta); plane_box_corner<5>(o, b, delta);
    plane_box_corner<6>(o, b, delta); plane_box_corner<7>(o, b, delta);
}

__device__ __forceinline__ void np_box_sphere(NOut& o, const Shp& bx, V3 c, float r, float delta) {
    V3 l = mulTv(bx.R, c - bx.c);
    V3 q = l;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float v = comp(l, i), h = dim(bx, i);
        setc(q, i, v < -h ? -h : (v > h ? h : v));
    }
    V3 dl = l - q;
    float d2 = dot3(dl, dl);
    if (d2 > 0.0f) {
        o.decision = 0;
        float dist = sqrtf(d2);
        V3 n = mulv(bx.R, (1.0f / dist) * dl);
        emit<0>(o, bx.c + mulv(bx.R, q), c - r * n, n, dist - r, delta);
    } else {
        int best = 0;
        float bd = bx.d[0] - fabsf(l.x);
#pragma unroll
        for (int i = 1; i < 3; ++i) {
            float di = dim(bx, i) - fabsf(comp(l, i));
            if (di < bd) { bd = di; best = i; }
        }
        float sg = comp(l, best) >= 0.0f ? 1.0f : -1.0f;
        V3 nl = v3(0.0f, 0.0f, 0.0f);
        setc(nl, best, sg);
        V3 n = mulv(bx.R, nl);
        V3 face = l;
        setc(face, best, sg * dim(bx, best));
        o.decision = 1 + best;
        emit<0>(o, bx.c + mulv(bx.R, face), c - r * n, n, -bd - r, delta);
    }
}

__device__ __forceinline__ float box_ext(const Shp& b, V3 L) {
    return (b.d[0] * fabsf(dot3(colm(b.R, 0), L)) + b.d[1] * fabsf(dot3(colm(b.R, 1), L))) +
           b.d[2] * fabsf(dot3(colm(b.R, 2), L));
}
__device__ __forceinline__ float tie_tol(float s, float hmin) { return 0.05f * fabsf(s) + 0.01f * hmin; }

__device__ __forceinline__ void clip_slab(V3 p0, V3 p1, V3 c, V3 a, float h, float& t0, float& t1) {
    float u0 = dot3(p0 - c, a), du = dot3(p1 - p0, a);
    if (fabsf(du) < 1e-12f) {
        if (u0 > h || u0 < -h) { t0 = 1.0f; t1 = 0.0f; }
        return;
    }
    float ta = (-h - u0) / du, tb = (h - u0) / du;
    if (ta > tb) { float tmp = ta; ta = tb; tb = tmp; }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
}

// A separating-axis candidate kept while scanning the axes in order: first strictly larger
// separation wins, exactly as an argmax over the axis list.
struct AxisBest {
    int k;
    float s;
    V3 L;
};

__device__ __forceinline__ void np_box_capsule(NOut& o, const Shp& bx, const Shp& cp, float delta) {
    V3 P0 = cp.p0(), P1 = cp.p1(), u = colm(cp.R, 2);
    float rc = cp.d[0], hl = cp.d[1];
    V3 dc = cp.c - bx.c;
    // face axes 0..2 and axis x edge axes 3..5; track the best face, the best valid edge and
    // the largest valid separation
    AxisBest bf{0, 0.0f, v3(0, 0, 0)}, be{-1, 0.0f, v3(0, 0, 0)};
    float smax = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        V3 L = colm(bx.R, i);
        if (dot3(L, dc) < 0.0f) L = -L;
        float sep = dot3(dc, L) - hl * fabsf(dot3(u, L)) - dim(bx, i) - rc;
        if (i == 0 || sep > bf.s) bf = AxisBest{i, sep, L};
        if (i == 0 || sep > smax) smax = sep;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        V3 L = cross3(u, colm(bx.R, i));
        float l = len3(L);
        if (l >= 1e-6f) {
            L = (1.0f / l) * L;
            if (dot3(L, dc) < 0.0f) L = -L;
            float sep = dot3(dc, L) - hl * fabsf(dot3(u, L)) - box_ext(bx, L) - rc;
            if (be.k < 0 || sep > be.s) be = AxisBest{3 + i, sep, L};
            if (sep > smax) smax = sep;
        }
    }
    float hmin = fminf(fminf(bx.d[0], bx.d[1]), fminf(bx.d[2], rc));
    AxisBest best = bf;
    if (be.k >= 0 && be.s > bf.s + tie_tol(bf.s, hmin)) best = be;
    o.decision = best.k;
    if (smax >= delta) return;
    if (best.k < 3) {
        int i = best.k;
        V3 nr = best.L;
        int j1 = (i + 1) % 3, j2 = (i + 2) % 3;
        float t0 = 0.0f, t1 = 1.0f;
        clip_slab(P0, P1, bx.c, axis(bx, j1), dim(bx, j1), t0, t1);
        clip_slab(P0, P1, bx.c, axis(bx, j2), dim(bx, j2), t0, t1);
        const float di = dim(bx, i);
        if (t0 <= t1) {
            {
                V3 C = P0 + t0 * (P1 - P0);
                float above = dot3(C - bx.c, nr) - di;
                emit<0>(o, C - above * nr, C - rc * nr, nr, above - rc, delta);
            }
            if (t1 > t0) {
                V3 C = P0 + t1 * (P1 - P0);
                float above = dot3(C - bx.c, nr) - di;
                emit<1>(o, C - above * nr, C - rc * nr, nr, above - rc, delta);
            }
        } else {
            o.decision = 6 + i;
            float bestd = 1e30f;
            V3 bs = v3(0.0f, 0.0f, 0.0f), be2 = v3(0.0f, 0.0f, 0.0f);
            V3 fc = bx.c + di * nr;
            const V3 a1 = axis(bx, j1), a2 = axis(bx, j2);
            const float h1 = dim(bx, j1), h2 = dim(bx, j2);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                V3 ca = vsel(k < 2, a1, a2), co = vsel(k < 2, a2, a1);     // along, other
                float ha = k < 2 ? h1 : h2, ho = k < 2 ? h2 : h1;
                float sg = (k & 1) ? 1.0f : -1.0f;
                V3 ec = fc + (sg * ho) * co;
                V3 e0 = ec - ha * ca, e1 = ec + ha * ca;
                float s, t;
                seg_seg(P0, P1, e0, e1, s, t);
                V3 cs = P0 + s * (P1 - P0), ce = e0 + t * (e1 - e0);
                V3 dd = cs - ce;
                float d2 = dot3(dd, dd);
                if (d2 < bestd) { bestd = d2; bs = cs; be2 = ce; }
            }
            float dist = sqrtf(bestd);
            V3 n = dist > 1e-9f ? (1.0f / dist) * (bs - be2) : nr;
            emit<0>(o, be2, bs - rc * n, n, dist - rc, delta);
        }
    } else {
        int i = best.k - 3;
        V3 L = best.L;
        V3 ec = bx.c;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            float dj = dot3(colm(bx.R, j), L);
            ec = ec + ((dj >= 0.0f ? 1.0f : -1.0f) * dim(bx, j)) * colm(bx.R, j);
        }
        V3 e0 = ec - dim(bx, i) * axis(bx, i), e1 = ec + dim(bx, i) * axis(bx, i);
        float s, t;
        seg_seg(P0, P1, e0, e1, s, t);
        V3 cs = P0 + s * (P1 - P0), ce = e0 + t * (e1 - e0);
        emit<0>(o, ce, cs - rc * L, L, dot3(cs - ce, L) - rc, delta);
    }
}

// Polygon of at most N vertices held in registers.
template <int N>
struct Poly {
    V3 v[N];
    int n;
};
// Write x at position `at` of a register polygon (a select per slot).
template <int N>
__device__ __forceinline__ void poly_put(Poly<N>& P, int at, V3 x) {
#pragma unroll
    for (int j = 0; j < N; ++j)
        if (j == at) P.v[j] = x;
}
// Sutherland-Hodgman step: keep the part of `in` with dot(x, a) <= off.  Walking the edges in
// order, a vertex inside is kept and an edge crossing the plane adds its crossing point (the
// output is capped at 8 vertices).  `ok` turns false if the output would outgrow NO slots, in
// which case the caller redoes the clip with 8-vertex polygons.
template <int NI, int NO>
__device__ __forceinline__ void clip_step(const Poly<NI>& in, V3 a, float off, Poly<NO>& out, bool& ok) {
    out.n = 0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        if (k < in.n) {
            V3 p = in.v[k];
            V3 q = vsel(k + 1 < in.n, in.v[k + 1 < NI ? k + 1 : 0], in.v[0]);
            float dp = dot3(p, a) - off, dq = dot3(q, a) - off;
            if (dp <= 0.0f && out.n < 8) {
                if (out.n < NO) poly_put(out, out.n, p); else ok = false;
                out.n++;
            }
            if (((dp < 0.0f && dq > 0.0f) || (dp > 0.0f && dq < 0.0f)) && out.n < 8) {
                float t = dp / (dp - dq);
                if (out.n < NO) poly_put(out, out.n, p + t * (q - p)); else ok = false;
                out.n++;
            }
        }
    }
    if (out.n > NO) out.n = NO;
}

// The incident face (4 vertices) clipped against the reference face's four side planes; first
// with slots for a convex input (one more vertex per plane), and only if a clip would outgrow
// them (a degenerate, numerically non-convex case) again with 8 slots throughout.
__device__ __forceinline__ void clip_face(const V3 q[4], V3 a1, float o1p, float o1m, V3 a2, float o2p, float o2m,
                                          Poly<8>& res) {
    bool ok = true;
    Poly<4> p4;
    p4.v[0] = q[0]; p4.v[1] = q[1]; p4.v[2] = q[2]; p4.v[3] = q[3]; p4.n = 4;
    Poly<5> p5; Poly<6> p6; Poly<7> p7;
    clip_step(p4, a1, o1p, p5, ok);
    clip_step(p5, -a1, o1m, p6, ok);
    clip_step(p6, a2, o2p, p7, ok);
    clip_step(p7, -a2, o2m, res, ok);
    if (!ok) {
        Poly<8> x, y;
        x.n = 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) x.v[j] = q[j];
#pragma unroll
        for (int j = 4; j < 8; ++j) x.v[j] = v3(0, 0, 0);
        bool dummy = true;
        clip_step(x, a1, o1p, y, dummy);
        clip_step(y, -a1, o1m, x, dummy);
        clip_step(x, a2, o2p, y, dummy);
        clip_step(y, -a2, o2m, res, dummy);
    }
}

template <int K>
__device__ __forceinline__ void emit_face_point(NOut& o, const Poly<8>& P, const Shp& Rf, V3 nref, float dri, V3 nAB,
                                                bool refA, float delta) {
    if (K < P.n) {
        V3 p = P.v[K];
        float s = dot3(p - Rf.c, nref) - dri;
        V3 onref = p - s * nref;
        if (refA) emit<K>(o, onref, p, nAB, s, delta);
        else emit<K>(o, p, onref, nAB, s, delta);
    }
}

__device__ __forceinline__ void np_box_box(NOut& o, const Shp& A, const Shp& B, float delta) {
    V3 d = B.c - A.c;
    // axes: A faces 0..2, B faces 3..5, edge crosses 6..14 (skipped when degenerate)
    AxisBest fa{0, 0.0f, v3(0, 0, 0)}, fb{3, 0.0f, v3(0, 0, 0)}, fe{-1, 0.0f, v3(0, 0, 0)};
    float smax = 0.0f;
#pragma unroll
    for (int k = 0; k < 15; ++k) {
        V3 L;
        bool valid = true;
        if (k < 3) L = colm(A.R, k);
        else if (k < 6) L = colm(B.R, k - 3);
        else {
            L = cross3(colm(A.R, (k - 6) / 3), colm(B.R, (k - 6) % 3));
            float l = len3(L);
            valid = l >= 1e-6f;
            L = (1.0f / l) * L;
        }
        if (valid) {
            if (dot3(L, d) < 0.0f) L = -L;
            float sep = dot3(d, L) - box_ext(A, L) - box_ext(B, L);
            if (k < 3) { if (k == 0 || sep > fa.s) fa = AxisBest{k, sep, L}; }
            else if (k < 6) { if (k == 3 || sep > fb.s) fb = AxisBest{k, sep, L}; }
            else if (fe.k < 0 || sep > fe.s) fe = AxisBest{k, sep, L};
            if (k == 0 || sep > smax) smax = sep;
        }
    }
    float hmin = fminf(fminf(fminf(A.d[0], A.d[1]), fminf(A.d[2], B.d[0])), fminf(B.d[1], B.d[2]));
    AxisBest best = fb;
    if (fa.s > fb.s + tie_tol(fb.s, hmin)) best = fa;
    if (fe.k >= 0 && fe.s > best.s + tie_tol(best.s, hmin)) best = fe;
    o.decision = best.k;
    if (smax >= delta) return;
    if (best.k < 6) {
        const bool refA = best.k < 3;
        const Shp Rf = pick(refA, A, B);
        const Shp In = pick(refA, B, A);
        const int ri = refA ? best.k : best.k - 3;
        V3 nref = vsel(refA, best.L, -best.L);
        int ii = 0;
        float bd = fabsf(dot3(colm(In.R, 0), nref));
#pragma unroll
        for (int j = 1; j < 3; ++j) {
            float dj = fabsf(dot3(colm(In.R, j), nref));
            if (dj > bd) { bd = dj; ii = j; }
        }
        const V3 ai = axis(In, ii);
        float sgn = dot3(ai, nref) >= 0.0f ? -1.0f : 1.0f;
        V3 fcen = In.c + (sgn * dim(In, ii)) * ai;
        int u = (ii + 1) % 3, v = (ii + 2) % 3;
        V3 U = dim(In, u) * axis(In, u), Wv = dim(In, v) * axis(In, v);
        V3 q[4] = {fcen + U + Wv, fcen - U + Wv, fcen - U - Wv, fcen + U - Wv};
        int r1 = (ri + 1) % 3, r2 = (ri + 2) % 3;
        V3 a1 = axis(Rf, r1), a2 = axis(Rf, r2);
        const float h1 = dim(Rf, r1), h2 = dim(Rf, r2);
        Poly<8> P;
        clip_face(q, a1, dot3(Rf.c, a1) + h1, -dot3(Rf.c, a1) + h1, a2, dot3(Rf.c, a2) + h2, -dot3(Rf.c, a2) + h2, P);
        V3 nAB = vsel(refA, nref, -nref);
        const float dri = dim(Rf, ri);
        emit_face_point<0>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<1>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<2>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<3>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<4>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<5>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<6>(o, P, Rf, nref, dri, nAB, refA, delta);
        emit_face_point<7>(o, P, Rf, nref, dri, nAB, refA, delta);
    } else {
        int ia = (best.k - 6) / 3, ib = (best.k - 6) % 3;
        V3 L = best.L;
        V3 ca = A.c, cb = B.c;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (j != ia) { float dj = dot3(colm(A.R, j), L); ca = ca + ((dj >= 0.0f ? 1.0f : -1.0f) * dim(A, j)) * colm(A.R, j); }
            if (j != ib) { float dj = dot3(colm(B.R, j), L); cb = cb + ((dj >= 0.0f ? -1.0f : 1.0f) * dim(B, j)) * colm(B.R, j); }
        }
        V3 a0 = ca - dim(A, ia) * axis(A, ia), a1 = ca + dim(A, ia) * axis(A, ia);
        V3 b0 = cb - dim(B, ib) * axis(B, ib), b1 = cb + dim(B, ib) * axis(B, ib);
        float s, t;
        seg_seg(a0, a1, b0, b1, s, t);
        V3 pa = a0 + s * (a1 - a0), pb = b0 + t * (b1 - b0);
        emit<0>(o, pa, pb, L, dot3(pb - pa, L), delta);
    }
}

__device__ __forceinline__ void np_capsule_capsule(NOut& o, const Shp& A, const Shp& B, float delta) {
    V3 a0 = A.p0(), a1 = A.p1(), b0 = B.p0(), b1 = B.p1();
    V3 d1 = a1 - a0, d2 = b1 - b0;
    V3 cr = cross3(d1, d2);
    if (dot3(cr, cr) < 1e-6f * dot3(d1, d1) * dot3(d2, d2)) {
        float dd = dot3(d1, d1);
        float s0 = dot3(b0 - a0, d1) / dd, s1 = dot3(b1 - a0, d1) / dd;
        float lo = fmaxf(0.0f, fminf(s0, s1)), hi = fminf(1.0f, fmaxf(s0, s1));
        if (lo < hi) {
            o.decision = 1;
            {
                V3 pa = a0 + lo * d1;
                float t = seg_point(b0, b1, pa);
                np_sphere_sphere<0>(o, pa, A.d[0], b0 + t * d2, B.d[0], delta);
            }
            {
                V3 pa = a0 + hi * d1;
                float t = seg_point(b0, b1, pa);
                np_sphere_sphere<1>(o, pa, A.d[0], b0 + t * d2, B.d[0], delta);
            }
            return;
        }
    }
    o.decision = 0;
    float s, t;
    seg_seg(a0, a1, b0, b1, s, t);
    np_sphere_sphere<0>(o, a0 + s * d1, A.d[0], b0 + t * d2, B.d[0], delta);
}

__device__ __forceinline__ void np_flip(NOut& o) {
#pragma unroll
    for (int k = 0; k < 2; ++k) o.pt[k].n = -o.pt[k].n;   // the flipped generators fill slots 0..1
}

__device__ __forceinline__ void np_pair(NOut& o, const Shp& A, const Shp& B, float delta) {
    int ta = A.type, tb = B.type;
    if (ta == 0 && tb == 0) { np_sphere_sphere<0>(o, A.c, A.d[0], B.c, B.d[0], delta); return; }
    if (ta == 0 && tb == 1) {
        float t = seg_point(B.p0(), B.p1(), A.c);
        np_sphere_sphere<0>(o, A.c, A.d[0], B.p0() + t * (B.p1() - B.p0()), B.d[0], delta);
        return;
    }
    if (ta == 1 && tb == 0) {
        float t = seg_point(A.p0(), A.p1(), B.c);
        np_sphere_sphere<0>(o, A.p0() + t * (A.p1() - A.p0()), A.d[0], B.c, B.d[0], delta);
        return;
    }
    if (ta == 1 && tb == 1) { np_capsule_capsule(o, A, B, delta); return; }
    if (ta == 2 && tb == 0) { np_box_sphere(o, A, B.c, B.d[0], delta); return; }
    if (ta == 0 && tb == 2) { np_box_sphere(o, B, A.c, A.d[0], delta); np_flip(o); return; }
    if (ta == 2 && tb == 1) { np_box_capsule(o, A, B, delta); return; }
    if (ta == 1 && tb == 2) { np_box_capsule(o, B, A, delta); np_flip(o); return; }
    np_box_box(o, A, B, delta);
}

__device__ __forceinline__ void np_plane(NOut& o, const Shp& B, float delta) {
    if (B.type == 0) np_plane_sphere<0>(o, B.c, B.d[0], delta);
    else if (B.type == 1) { np_plane_sphere<0>(o, B.p0(), B.d[0], delta); np_plane_sphere<1>(o, B.p1(), B.d[0], delta); }
    else np_plane_box(o, B, delta);
}

// <= 4 points: deepest; farthest from it; largest triangle; most area added outside the
// triangle; first point of the list on ties; kept points in their original order.  The list is
// the valid slots in slot order; `used` marks slots.
__device__ __forceinline__ void reduce4(NOut& o) {
    if (n_points(o) <= 4) return;
    const uint32_t valid = o.mask;
    // deepest
    int k0 = __ffs(valid) - 1;
    float s0 = 0.0f;
    V3 p0 = v3(0, 0, 0);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k == k0) { s0 = o.pt[k].s; p0 = o.pt[k].p; }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (((valid >> k) & 1) && o.pt[k].s < s0) { k0 = k; s0 = o.pt[k].s; p0 = o.pt[k].p; }
    uint32_t used = 1u << k0;
    // farthest from the deepest (starting from the first unused point)
    int k1 = __ffs(valid & ~used) - 1;
    float b1 = -1.0f;
    V3 p1 = v3(0, 0, 0);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k == k1) p1 = o.pt[k].p;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!((valid & ~used) >> k & 1)) continue;
        V3 dd = o.pt[k].p - p0;
        float v = dot3(dd, dd);
        if (v > b1) { b1 = v; k1 = k; p1 = o.pt[k].p; }
    }
    used |= 1u << k1;
    // largest triangle with the first two
    int k2 = __ffs(valid & ~used) - 1;
    float b2 = -1.0f;
    V3 p2 = v3(0, 0, 0);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k == k2) p2 = o.pt[k].p;
    V3 e01 = p1 - p0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!((valid & ~used) >> k & 1)) continue;
        V3 cc = cross3(e01, o.pt[k].p - p0);
        float v = dot3(cc, cc);
        if (v > b2) { b2 = v; k2 = k; p2 = o.pt[k].p; }
    }
    used |= 1u << k2;
    V3 nt = cross3(e01, p2 - p0);
    // most area added outside the triangle
    int k3 = __ffs(valid & ~used) - 1;
    float b3 = -1e30f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!((valid & ~used) >> k & 1)) continue;
        float bestv = -1e30f;
        {
            float v = -dot3(cross3(p1 - p0, o.pt[k].p - p0), nt);
            if (v > bestv) bestv = v;
        }
        {
            float v = -dot3(cross3(p2 - p1, o.pt[k].p - p1), nt);
            if (v > bestv) bestv = v;
        }
        {
            float v = -dot3(cross3(p0 - p2, o.pt[k].p - p2), nt);
            if (v > bestv) bestv = v;
        }
        if (bestv > b3) { b3 = bestv; k3 = k; }
    }
    used |= 1u << k3;
    o.mask = used;
}

// Move the (at most 4 after reduce4) points of the list into slots 0.. in list order.
__device__ __forceinline__ void compact4(NOut& o) {
    Pt out[4] = {o.pt[0], o.pt[1], o.pt[2], o.pt[3]};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!((o.mask >> k) & 1)) continue;
        const int r = __popc(o.mask & ((1u << k) - 1));
#pragma unroll
        for (int j = 0; j < 4 && j <= k; ++j)
            if (r == j) out[j] = o.pt[k];
    }
    const int n = min(__popc(o.mask), 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) o.pt[j] = out[j];
    o.mask = (1u << n) - 1;
}

// Duff et al. 2017 orthonormal basis: t1 for unit n (t2 = n x t1).
__device__ __forceinline__ V3 onb_t1(V3 n) {
    float sg = copysignf(1.0f, n.z);
    float a = -1.0f / (sg + n.z);
    float b = n.x * n.y * a;
    return v3(1.0f + sg * n.x * n.x * a, sg * b, -sg * n.x);
}

// ----------------------------------------------------------------------------- LDS body helpers
__device__ __forceinline__ float invm_of(const EnvCtx& c, int i) { return i < 0 ? 0.0f : body_rec(c, i)[B_IM]; }
__device__ __forceinline__ V3 v_of(const EnvCtx& c, int i) { return i < 0 ? v3(0, 0, 0) : ldv(c, i); }
__device__ __forceinline__ V3 w_of(const EnvCtx& c, int i) { return i < 0 ? v3(0, 0, 0) : ldw(c, i); }

__device__ __forceinline__ float eff_mass(const EnvCtx& c, int a, int b, V3 rA, V3 rB, V3 x) {
    float k = invm_of(c, a) + invm_of(c, b);
    if (a >= 0) { V3 cr = cross3(rA, x); k += dot3(cr, muls(load_iw(c, a), cr)); }
    if (b >= 0) { V3 cr = cross3(rB, x); k += dot3(cr, muls(load_iw(c, b), cr)); }
    return k > 0.0f ? 1.0f / k : 0.0f;
}

__device__ __forceinline__ Shp shape_of(const EnvCtx& c, int i, V3 centre) {
    Shp s;
    const Lay& l = c.lay;
    s.type = iptr(c.L + l.SH)[i] & 0xFF;
    s.c = centre;
    s.R = rotm(ldp4(c, i, P_Q0));
    s.d[0] = c.L[l.DIM + i]; s.d[1] = c.L[l.DIM + l.n + i]; s.d[2] = c.L[l.DIM + 2 * l.n + i];
    return s;
}

// ----------------------------------------------------------------------------- compound parts
// A compound body holds its table index in dim0; its record (HBM, shared by every env of the
// batch and read through the caches) lists its primitive parts with their body-frame poses.
__device__ __forceinline__ bool is_compound(const EnvCtx& c, int i) {
    return (iptr(c.L + c.lay.SH)[i] & 0xFF) == SHAPE_COMPOUND;
}
__device__ __forceinline__ const float* comp_rec(const EnvCtx& c, int i) {
    return c.bd->comp + size_t(int(c.L[c.lay.DIM + i])) * COMP_WORDS;
}
__device__ __forceinline__ int n_parts(const EnvCtx& c, int i) {
    return is_compound(c, i) ? gldi(reinterpret_cast<const int*>(comp_rec(c, i))) : 1;
}
// Part k of body i with the body's centre at `centre` (pair frame): the body itself, or a
// compound's part at centre + R c_k with rotation R(q q_k), q the step-start orientation.
__device__ __forceinline__ Shp part_of(const EnvCtx& c, int i, int k, V3 centre) {
    if (!is_compound(c, i)) return shape_of(c, i, centre);
    const float4* P = reinterpret_cast<const float4*>(comp_rec(c, i) + 4 + 12 * k);
    const float4 r0 = gld4(P), r1 = gld4(P + 1), r2 = gld4(P + 2);
    const Qt q = ldp4(c, i, P_Q0);
    Shp s;
    s.type = __float_as_int(r0.x);
    s.d[0] = r0.y; s.d[1] = r0.z; s.d[2] = r0.w;
    s.c = centre + mulv(rotm(q), v3(r1.x, r1.y, r1.z));
    s.R = rotm(qmul(q, Qt{r1.w, r2.x, r2.y, r2.z}));
    return s;
}

// ----------------------------------------------------------------------------- manifold block
// Rows are records (array of structures): a manifold's 23 words and a point's 14 words are
// contiguous, so a lane's row loads share one address and pair up into wide LDS reads.
constexpr int M_WORDS = 23, R_WORDS = 14;
__device__ __forceinline__ float mf(const EnvCtx& c, int plane, int m) { return c.L[c.lay.MAN + m * M_WORDS + plane]; }
__device__ __forceinline__ float& mfr(const EnvCtx& c, int plane, int m) { return c.L[c.lay.MAN + m * M_WORDS + plane]; }
__device__ __forceinline__ V3 mf3(const EnvCtx& c, int plane, int m) {
    return v3(mf(c, plane, m), mf(c, plane + 1, m), mf(c, plane + 2, m));
}
__device__ __forceinline__ float& pr(const EnvCtx& c, int plane, int k) { return c.L[c.lay.PT + k * R_WORDS + plane]; }
__device__ __forceinline__ V3 pr3(const EnvCtx& c, int plane, int k) {
    return v3(pr(c, plane, k), pr(c, plane + 1, k), pr(c, plane + 2, k));
}

__device__ __forceinline__ void man_header(const EnvCtx& c, int m, int& a, int& b, int& first, int& cnt) {
    int ab = iptr(c.L + c.lay.MAN + m * M_WORDS)[M_AB];
    int fc = iptr(c.L + c.lay.MAN + m * M_WORDS)[M_FC];
    a = (ab & 0xFF) == 0xFF ? -1 : (ab & 0xFF);
    b = (ab >> 8) & 0xFF;
    first = fc & 0xFFFF;
    cnt = fc >> 16;
}

// A block owns its dynamic bodies for the duration of its colour, so a lane keeps the two bodies
// of its block in registers for the whole block solve and writes them back once.
struct BodyR {
    V3 v, w;
    float im;
    S6 I;
    bool dyn;
};
struct PoseR {
    V3 dx;
    Qt dq;
};
__device__ __forceinline__ BodyR load_body(const EnvCtx& c, int i) {
    BodyR r;
    if (i < 0) {
        r.v = v3(0, 0, 0); r.w = v3(0, 0, 0); r.im = 0.0f; r.I = S6{0, 0, 0, 0, 0, 0}; r.dyn = false;
        return r;
    }
    const int n = c.lay.n;
    r.v = ldv(c, i);
    r.w = ldw(c, i);
    r.im = body_rec(c, i)[B_IM];
    r.I = load_iw(c, i);
    r.dyn = is_dyn(c, i);
    return r;
}
__device__ __forceinline__ void store_body(const EnvCtx& c, int i, const BodyR& r) {
    if (!r.dyn) return;
    const int n = c.lay.n;
    stv(c, i, r.v);
    stw(c, i, r.w);
}
__device__ __forceinline__ PoseR load_pose(const EnvCtx& c, int i) {
    if (i < 0) return PoseR{v3(0, 0, 0), Qt{1.0f, 0.0f, 0.0f, 0.0f}};
    return PoseR{ldp3(c, i, P_DX), ldp4(c, i, P_DQ)};
}
// -P on A at arm rA, +P on B at arm rB (dynamic bodies only).
__device__ __forceinline__ void imp_lin(BodyR& A, BodyR& B, V3 rA, V3 rB, V3 P) {
    if (A.dyn) { A.v = A.v - A.im * P; A.w = A.w - muls(A.I, cross3(rA, P)); }
    if (B.dyn) { B.v = B.v + B.im * P; B.w = B.w + muls(B.I, cross3(rB, P)); }
}
__device__ __forceinline__ void imp_ang(BodyR& A, BodyR& B, V3 L) {
    if (A.dyn) A.w = A.w - muls(A.I, L);
    if (B.dyn) B.w = B.w + muls(B.I, L);
}
__device__ __forceinline__ V3 relv(const BodyR& A, const BodyR& B, bool has_a, V3 rA, V3 rB) {
    V3 vb = B.v + cross3(B.w, rB);
    V3 va = has_a ? A.v + cross3(A.w, rA) : v3(0, 0, 0);
    return vb - va;
}
// Displacement of the body-fixed point x0 + r since the step start: dx + R(dq) r - r.
__device__ __forceinline__ V3 disp(const PoseR& p, V3 r) {
    V3 u = v3(p.dq.x, p.dq.y, p.dq.z);
    V3 ur = cross3(u, r);
    return p.dx + (2.0f * p.dq.w) * ur + 2.0f * cross3(u, ur);
}

__device__ __forceinline__ V3 rel_vel(const EnvCtx& c, int a, int b, V3 rA, V3 rB) {
    V3 vb = v_of(c, b) + cross3(w_of(c, b), rB);
    V3 va = a >= 0 ? v_of(c, a) + cross3(w_of(c, a), rA) : v3(0, 0, 0);
    return vb - va;
}

__device__ __forceinline__ void manifold_restitution(const EnvCtx& c, int m) {
    const BatchDev& bd = *c.bd;
    int a, b, first, cnt;
    man_header(c, m, a, b, first, cnt);
    const bool has_a = a >= 0;
    BodyR A = load_body(c, a), B = load_body(c, b);
    bool any = false;
    for (int k = first; k < first + cnt; ++k) {
        float vpre = pr(c, R_VN, k);
        float old = pr(c, R_LN, k);
        if (!(vpre < -bd.bounce && old > 0.0f)) continue;
        any = true;
        V3 rA = pr3(c, R_RA, k), rB = pr3(c, R_RB, k), n = pr3(c, R_N, k);
        float vn = dot3(relv(A, B, has_a, rA, rB), n);
        float dl = -pr(c, R_MN, k) * (vn + mf(c, M_REST, m) * vpre);
        float nl = fmaxf(old + dl, 0.0f);
        pr(c, R_LN, k) = nl;
        imp_lin(A, B, rA, rB, (nl - old) * n);
    }
    if (any) {
        store_body(c, a, A);
        store_body(c, b, B);
    }
}

// ----------------------------------------------------------------------------- joint block
// Arctangent of the drive angle from correctly rounded +, *, / and sqrt only: two half-angle
// steps tan(a/2) = t / (1 + sqrt(1 + t^2)) take t in [0, 1] below tan(pi/16), then the
// alternating series u - u^3/3 + ... - u^15/15 (Horner) and a factor 4.
__device__ __forceinline__ float atan_01(float t) {
    float u = t / (1.0f + sqrtf(1.0f + t * t));
    u = u / (1.0f + sqrtf(1.0f + u * u));
    float u2 = u * u;
    float p = 1.0f / 15.0f;
    p = 1.0f / 13.0f - u2 * p;
    p = 1.0f / 11.0f - u2 * p;
    p = 1.0f / 9.0f - u2 * p;
    p = 1.0f / 7.0f - u2 * p;
    p = 1.0f / 5.0f - u2 * p;
    p = 1.0f / 3.0f - u2 * p;
    p = 1.0f - u2 * p;
    return 4.0f * (u * p);
}
// atan2(y, w) for w >= 0, via atan(t) = pi/2 - atan(1/t) above the diagonal.
__device__ __forceinline__ float atan2_w(float y, float w) {
    float ay = fabsf(y);
    float a;
    if (ay <= w) a = w > 0.0f ? atan_01(ay / w) : 0.0f;
    else a = 3.14159265358979323846f / 2.0f - atan_01(w / ay);
    return y < 0.0f ? -a : a;
}

// Frames of a joint from the current poses: arms rA = R(qA) aA, rB = R(qB) aB, the axes of the
// parent's joint frame and the anchors' separation d = (xB + rB) - (xA + rA); a prismatic
// joint's parent arm reaches the child anchor (rA + d).
struct JFrame { int a, b; V3 rA, rB, zA, b1, b2, d; Qt qa, qb; };
__device__ __forceinline__ float* jrec(const EnvCtx& c, int j) { return c.L + c.lay.JNT + J_WORDS * j; }
__device__ __forceinline__ bool jprism(const float* J) {
    return (reinterpret_cast<const int*>(J)[J_TYP] & 0xFF) == JOINT_PRISMATIC;
}
__device__ __forceinline__ bool jlimited(const float* J) { return (reinterpret_cast<const int*>(J)[J_TYP] >> 8) & 1; }
__device__ __forceinline__ V3 x_of(const EnvCtx& c, int i) {
    return i < 0 ? v3(0, 0, 0) : ldp3(c, i, P_X0) + ldp3(c, i, P_DX);
}
__device__ __forceinline__ Qt qc_of(const EnvCtx& c, int i) {
    return i < 0 ? Qt{1.0f, 0.0f, 0.0f, 0.0f} : ldp4(c, i, P_QC);
}

__device__ __forceinline__ JFrame joint_frame(const EnvCtx& c, int j) {
    const float* J = jrec(c, j);
    JFrame f;
    f.a = reinterpret_cast<const int*>(J)[J_PA];
    f.b = reinterpret_cast<const int*>(J)[J_CH];
    f.qa = qc_of(c, f.a);
    f.qb = qc_of(c, f.b);
    f.rA = mulv(rotm(f.qa), v3(J[J_AA], J[J_AA + 1], J[J_AA + 2]));
    f.rB = mulv(rotm(f.qb), v3(J[J_AB], J[J_AB + 1], J[J_AB + 2]));
    M3 Ra = rotm(qmul(f.qa, Qt{J[J_QA], J[J_QA + 1], J[J_QA + 2], J[J_QA + 3]}));
    f.zA = colm(Ra, 2); f.b1 = colm(Ra, 0); f.b2 = colm(Ra, 1);
    f.d = (x_of(c, f.b) + f.rB) - (x_of(c, f.a) + f.rA);
    if (jprism(J)) f.rA = f.rA + f.d;
    return f;
}

// Quantities of a joint that depend only on the poses, the frozen inertias and the joint
// record, so they stay fixed through the colour sweeps of a substep (poses change only when the
// substep integrates): anchors and frame axes, the adjugate and determinant of the point block,
// the position error, the angular block and its errors, the drive's softness terms.  joint_prep
// stores them once per substep; the warm start and joint_solve read them.  Same operations in the same
// order as computing them inside every visit.
// A revolute joint's 3x3 block is its point block (ADJ, DET, position error CP = d) and its 2x2
// block the axis alignment (K11..DET2, errors C1, C2); a prismatic joint's 3x3 block is its
// rotation lock (K = IA + IB, error CP = 2 vec(q_rel) in the world) and its 2x2 block the rows
// across the slide axis (errors b1 . d, b2 . d).  Limits: MLIM = 1 / k of the free axis and the
// gaps SLO = x - lower, SHI = upper - x.
enum { JI_RA = 0, JI_RB = 3, JI_ZA = 6, JI_B1 = 9, JI_B2 = 12, JI_ADJ = 15, JI_DET = 24, JI_CP = 25, JI_C1 = 28,
       JI_C2 = 29, JI_K11 = 30, JI_K12 = 31, JI_K22 = 32, JI_DET2 = 33, JI_GAM = 34, JI_KG = 35, JI_BCH = 36,
       JI_MLIM = 37, JI_SLO = 38, JI_SHI = 39, JI_WORDS = 40 };
__device__ __forceinline__ float* jinv(const EnvCtx& c, int j) { return c.L + c.lay.JINV + JI_WORDS * j; }
__device__ __forceinline__ V3 jv3(const float* P, int o) { return v3(P[o], P[o + 1], P[o + 2]); }
__device__ __forceinline__ void jst3(float* P, int o, V3 v) { P[o] = v.x; P[o + 1] = v.y; P[o + 2] = v.z; }

// Adjugate (row-major) and determinant of a 3x3 matrix.
__device__ __forceinline__ void adj3(const float K[3][3], float* A9, float& det) {
    A9[0] = K[1][1] * K[2][2] - K[1][2] * K[2][1];
    A9[1] = K[0][2] * K[2][1] - K[0][1] * K[2][2];
    A9[2] = K[0][1] * K[1][2] - K[0][2] * K[1][1];
    A9[3] = K[1][2] * K[2][0] - K[1][0] * K[2][2];
    A9[4] = K[0][0] * K[2][2] - K[0][2] * K[2][0];
    A9[5] = K[0][2] * K[1][0] - K[0][0] * K[1][2];
    A9[6] = K[1][0] * K[2][1] - K[1][1] * K[2][0];
    A9[7] = K[0][1] * K[2][0] - K[0][0] * K[2][1];
    A9[8] = K[0][0] * K[1][1] - K[0][1] * K[1][0];
    det = K[0][0] * A9[0] + K[0][1] * A9[3] + K[0][2] * A9[6];
}

__device__ __forceinline__ void joint_prep(const EnvCtx& c, int j, float h) {
    JFrame f = joint_frame(c, j);
    const float* J = jrec(c, j);
    float* P = jinv(c, j);
    const int a = f.a, b = f.b;
    const bool prism = jprism(J);
    const S6 Ia = a >= 0 ? load_iw(c, a) : S6{0, 0, 0, 0, 0, 0};
    const S6 Ib = load_iw(c, b);
    const float ima = invm_of(c, a), imb = invm_of(c, b);
    jst3(P, JI_RA, f.rA); jst3(P, JI_RB, f.rB); jst3(P, JI_ZA, f.zA); jst3(P, JI_B1, f.b1); jst3(P, JI_B2, f.b2);
    const Qt qaf = qmul(f.qa, Qt{J[J_QA], J[J_QA + 1], J[J_QA + 2], J[J_QA + 3]});
    const Qt qbf = qmul(f.qb, Qt{J[J_QB], J[J_QB + 1], J[J_QB + 2], J[J_QB + 3]});
    if (!prism) {
        // point block: K = (mA^-1 + mB^-1) I - [rA]x IA [rA]x - [rB]x IB [rB]x, its adjugate and determinant
        float im = ima + imb;
        float K[3][3] = {{im, 0, 0}, {0, im, 0}, {0, 0, im}};
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (side == 0 && a < 0) continue;
            V3 r = vsel(side == 0, f.rA, f.rB);
            const S6& I = side == 0 ? Ia : Ib;
            float Im[3][3] = {{I.xx, I.xy, I.xz}, {I.xy, I.yy, I.yz}, {I.xz, I.yz, I.zz}};
            float Sx[3][3] = {{0, -r.z, r.y}, {r.z, 0, -r.x}, {-r.y, r.x, 0}};
            float SI[3][3];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) SI[p][q] = Sx[p][0] * Im[0][q] + Sx[p][1] * Im[1][q] + Sx[p][2] * Im[2][q];
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int q = 0; q < 3; ++q) K[p][q] -= SI[p][0] * Sx[0][q] + SI[p][1] * Sx[1][q] + SI[p][2] * Sx[2][q];
        }
        adj3(K, P + JI_ADJ, P[JI_DET]);
        jst3(P, JI_CP, f.d);
        // angular block: axis misalignment and the 2x2 block
        V3 zB = colm(rotm(qbf), 2);
        V3 zc = cross3(f.zA, zB);
        P[JI_C1] = dot3(f.b1, zc);
        P[JI_C2] = dot3(f.b2, zc);
        S6 Is{Ia.xx + Ib.xx, Ia.yy + Ib.yy, Ia.zz + Ib.zz, Ia.xy + Ib.xy, Ia.xz + Ib.xz, Ia.yz + Ib.yz};
        float k11 = dot3(f.b1, muls(Is, f.b1)), k12 = dot3(f.b1, muls(Is, f.b2)), k22 = dot3(f.b2, muls(Is, f.b2));
        P[JI_K11] = k11; P[JI_K12] = k12; P[JI_K22] = k22;
        P[JI_DET2] = k11 * k22 - k12 * k12;
    } else {
        // rotation lock: error 2 vec(q_rel) (q_rel.w >= 0) in the parent's joint frame, K = IA + IB
        Qt rel = qmul(Qt{qaf.w, -qaf.x, -qaf.y, -qaf.z}, qbf);
        if (rel.w < 0.0f) rel = Qt{-rel.w, -rel.x, -rel.y, -rel.z};
        V3 e = (2.0f * rel.x) * f.b1 + (2.0f * rel.y) * f.b2 + (2.0f * rel.z) * f.zA;
        float K[3][3] = {{Ia.xx + Ib.xx, Ia.xy + Ib.xy, Ia.xz + Ib.xz},
                         {Ia.xy + Ib.xy, Ia.yy + Ib.yy, Ia.yz + Ib.yz},
                         {Ia.xz + Ib.xz, Ia.yz + Ib.yz, Ia.zz + Ib.zz}};
        adj3(K, P + JI_ADJ, P[JI_DET]);
        jst3(P, JI_CP, e);
        // the child anchor on the slide line: rows along b1, b2 at the arms rA + d and rB
        const V3 cA1 = cross3(f.rA, f.b1), cA2 = cross3(f.rA, f.b2), cB1 = cross3(f.rB, f.b1), cB2 = cross3(f.rB, f.b2);
        const float im = ima + imb;
        const float k11 = (im + dot3(cA1, muls(Ia, cA1))) + dot3(cB1, muls(Ib, cB1));
        const float k12 = dot3(cA1, muls(Ia, cA2)) + dot3(cB1, muls(Ib, cB2));
        const float k22 = (im + dot3(cA2, muls(Ia, cA2))) + dot3(cB2, muls(Ib, cB2));
        P[JI_K11] = k11; P[JI_K12] = k12; P[JI_K22] = k22;
        P[JI_DET2] = k11 * k22 - k12 * k12;
        P[JI_C1] = dot3(f.b1, f.d);
        P[JI_C2] = dot3(f.b2, f.d);
    }
    // the free axis: drive (soft-row terms) and limits (effective mass, gaps)
    const float kp = J[J_KP], kd = J[J_KD];
    const bool drive = kp != 0.0f || kd != 0.0f, lim = jlimited(J);
    if (drive || lim) {
        const V3 ax = f.zA;
        float k, x;
        if (prism) {
            k = ima + imb;
            if (a >= 0) { V3 cc = cross3(f.rA, ax); k = k + dot3(cc, muls(Ia, cc)); }
            V3 cc = cross3(f.rB, ax);
            k = k + dot3(cc, muls(Ib, cc));
            x = dot3(ax, f.d);
        } else {
            k = dot3(ax, muls(Ib, ax)) + (a >= 0 ? dot3(ax, muls(Ia, ax)) : 0.0f);
            Qt rel = qmul(Qt{qaf.w, -qaf.x, -qaf.y, -qaf.z}, qbf);
            if (rel.w < 0.0f) rel = Qt{-rel.w, -rel.x, -rel.y, -rel.z};
            x = 2.0f * atan2_w(rel.z, rel.w);
        }
        if (drive) {
            float den = kd + h * kp;
            float gamma = 1.0f / (h * den);
            float beta_d = h * kp / den;
            float C = x - J[J_TG];
            if (!prism) {
                // wrap into (-pi, pi] with the exact IEEE remainder (non-finite stays non-finite)
                const float pi = 3.14159265358979323846f;
                C = remainderf(C, 2.0f * pi);
                if (C <= -pi) C += 2.0f * pi;
            }
            P[JI_GAM] = gamma;
            P[JI_KG] = k + gamma;
            P[JI_BCH] = beta_d * C / h;
        }
        if (lim) {
            P[JI_MLIM] = k > 0.0f ? 1.0f / k : 0.0f;
            P[JI_SLO] = x - J[J_LO];
            P[JI_SHI] = J[J_HI] - x;
        }
    }
}

// The two one-sided limit rows of a joint along its free axis (lower, then upper): speculative
// while the gap is open (bias gap / h), Baumgarte at the joint rate per step once closed (none in
// a velocity pass); accumulated impulses >= 0.
__device__ __forceinline__ void joint_limits(const EnvCtx& c, int j, bool prism, BodyR& A, BodyR& B, bool has_a, V3 rA,
                                             V3 rB, V3 ax, float h, float brate, bool vpass) {
    const float* P = jinv(c, j);
    float* J = jrec(c, j);
    const float m = P[JI_MLIM];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const float gap = side == 0 ? P[JI_SLO] : P[JI_SHI];
        const float bias = gap > 0.0f ? gap / h : (vpass ? 0.0f : brate * gap);
        float v = prism ? dot3(ax, relv(A, B, has_a, rA, rB)) : dot3(ax, B.w - A.w);
        if (side == 1) v = -v;
        const float old = J[J_LL + side];
        const float nl = fmaxf(old - m * (v + bias), 0.0f);
        const float dl = nl - old;
        J[J_LL + side] = nl;
        const float l = side == 0 ? dl : -dl;
        if (prism) imp_lin(A, B, rA, rB, l * ax);
        else imp_ang(A, B, l * ax);
    }
}

__device__ __forceinline__ void joint_solve(const EnvCtx& c, int j, float h, bool vpass) {
    const BatchDev& bd = *c.bd;
    const float* P = jinv(c, j);
    float* J = jrec(c, j);
    const int a = reinterpret_cast<const int*>(J)[J_PA], b = reinterpret_cast<const int*>(J)[J_CH];
    const bool prism = jprism(J);
    const V3 rA = jv3(P, JI_RA), rB = jv3(P, JI_RB);
    const float brate = vpass ? 0.0f : bd.beta_j / bd.dt;
    BodyR A = load_body(c, a), B = load_body(c, b);
    const bool has_a = a >= 0;
    // 3x3 block: revolute point block (linear at the arms), prismatic rotation lock (angular)
    {
        V3 C = jv3(P, JI_CP);
        V3 Cd = prism ? B.w - A.w : (B.v + cross3(B.w, rB)) - (A.v + cross3(A.w, rA));
        V3 rhs = Cd + brate * C;
        const float det = P[JI_DET];
        if (det != 0.0f) {
            const float* A9 = P + JI_ADJ;
            float id = 1.0f / det;
            V3 lam = v3(-(A9[0] * rhs.x + A9[1] * rhs.y + A9[2] * rhs.z) * id, -(A9[3] * rhs.x + A9[4] * rhs.y + A9[5] * rhs.z) * id,
                        -(A9[6] * rhs.x + A9[7] * rhs.y + A9[8] * rhs.z) * id);
            if (prism) {
                J[J_LA] += lam.x; J[J_LA + 1] += lam.y; J[J_LA + 2] += lam.z;
                imp_ang(A, B, lam);
            } else {
                J[J_LP] += lam.x; J[J_LP + 1] += lam.y; J[J_LP + 2] += lam.z;
                imp_lin(A, B, rA, rB, lam);
            }
        }
    }
    // 2x2 block: revolute axis alignment (angular about b1, b2), prismatic rows across the slide
    // axis (linear along b1, b2 at the arms)
    {
        const V3 b1 = jv3(P, JI_B1), b2 = jv3(P, JI_B2);
        float Cd1, Cd2;
        if (prism) {
            V3 vr = relv(A, B, has_a, rA, rB);
            Cd1 = dot3(b1, vr); Cd2 = dot3(b2, vr);
        } else {
            V3 dw = B.w - A.w;
            Cd1 = dot3(b1, dw); Cd2 = dot3(b2, dw);
        }
        const float k11 = P[JI_K11], k12 = P[JI_K12], k22 = P[JI_K22];
        float r1 = Cd1 + brate * P[JI_C1], r2 = Cd2 + brate * P[JI_C2];
        float det = P[JI_DET2];
        if (det != 0.0f) {
            float id = 1.0f / det;
            float l1 = -(k22 * r1 - k12 * r2) * id;
            float l2 = -(-k12 * r1 + k11 * r2) * id;
            if (prism) {
                J[J_LP] += l1; J[J_LP + 1] += l2;
                imp_lin(A, B, rA, rB, l1 * b1 + l2 * b2);
            } else {
                J[J_LA] += l1; J[J_LA + 1] += l2;
                imp_ang(A, B, l1 * b1 + l2 * b2);
            }
        }
    }
    // PD drive: soft row along the free axis
    const V3 ax = jv3(P, JI_ZA);
    float kp = J[J_KP], kd = J[J_KD];
    if (kp != 0.0f || kd != 0.0f) {
        float Cd = prism ? dot3(ax, relv(A, B, has_a, rA, rB)) : dot3(ax, B.w - A.w);
        float dl = -(Cd + P[JI_BCH] + P[JI_GAM] * J[J_LD]) / P[JI_KG];
        J[J_LD] += dl;
        if (prism) imp_lin(A, B, rA, rB, dl * ax);
        else imp_ang(A, B, dl * ax);
    }
    if (jlimited(J)) joint_limits(c, j, prism, A, B, has_a, rA, rB, ax, h, brate, vpass);
    store_body(c, a, A);
    store_body(c, b, B);
}

// A joint visit from values loaded ahead: everything joint_solve reads except the two bodies'
// velocities (the block's own accumulated impulses change only in its own visit, the rest only
// between substeps).  Used by the joint-only sweeps, where a lane's next joint is loaded at the
// end of the current entry.
struct JointPre {
    int a, b;
    V3 rA, rB, zA, b1, b2, CP, lp;
    float adj[9];
    float det, C1, C2, k11, k12, k22, det2, gam, kg, bch, kp, kd, la0, la1, la2, ld;
    float ima, imb;
    S6 Ia, Ib;
    bool da, db, prism, lim;
};
__device__ __forceinline__ void joint_prefetch(const EnvCtx& c, int j, JointPre& q) {
    const float* P = jinv(c, j);
    const float* J = jrec(c, j);
    q.a = reinterpret_cast<const int*>(J)[J_PA];
    q.b = reinterpret_cast<const int*>(J)[J_CH];
    q.prism = jprism(J);
    q.lim = jlimited(J);
    q.rA = jv3(P, JI_RA); q.rB = jv3(P, JI_RB); q.zA = jv3(P, JI_ZA); q.b1 = jv3(P, JI_B1); q.b2 = jv3(P, JI_B2);
    q.CP = jv3(P, JI_CP);
#pragma unroll
    for (int k = 0; k < 9; ++k) q.adj[k] = P[JI_ADJ + k];
    q.det = P[JI_DET]; q.C1 = P[JI_C1]; q.C2 = P[JI_C2];
    q.k11 = P[JI_K11]; q.k12 = P[JI_K12]; q.k22 = P[JI_K22]; q.det2 = P[JI_DET2];
    q.gam = P[JI_GAM]; q.kg = P[JI_KG]; q.bch = P[JI_BCH];
    q.kp = J[J_KP]; q.kd = J[J_KD];
    q.lp = v3(J[J_LP], J[J_LP + 1], J[J_LP + 2]); q.la0 = J[J_LA]; q.la1 = J[J_LA + 1]; q.la2 = J[J_LA + 2]; q.ld = J[J_LD];
    q.da = is_dyn(c, q.a); q.db = is_dyn(c, q.b);
    q.ima = invm_of(c, q.a); q.imb = invm_of(c, q.b);
    q.Ia = q.a >= 0 ? load_iw(c, q.a) : S6{0, 0, 0, 0, 0, 0};
    q.Ib = load_iw(c, q.b);
}
__device__ __forceinline__ void joint_solve_pre(const EnvCtx& c, int j, const JointPre& q, float brate, float h) {
    float* J = jrec(c, j);
    const int n = c.lay.n;
    const bool has_a = q.a >= 0;
    BodyR A, B;
    if (q.a >= 0) { A.v = ldv(c, q.a); A.w = ldw(c, q.a); }
    else { A.v = v3(0, 0, 0); A.w = v3(0, 0, 0); }
    B.v = ldv(c, q.b);
    B.w = ldw(c, q.b);
    A.im = q.ima; A.I = q.Ia; A.dyn = q.da;
    B.im = q.imb; B.I = q.Ib; B.dyn = q.db;
    {
        V3 Cd = q.prism ? B.w - A.w : (B.v + cross3(B.w, q.rB)) - (A.v + cross3(A.w, q.rA));
        V3 rhs = Cd + brate * q.CP;
        if (q.det != 0.0f) {
            float id = 1.0f / q.det;
            V3 lam = v3(-(q.adj[0] * rhs.x + q.adj[1] * rhs.y + q.adj[2] * rhs.z) * id,
                        -(q.adj[3] * rhs.x + q.adj[4] * rhs.y + q.adj[5] * rhs.z) * id,
                        -(q.adj[6] * rhs.x + q.adj[7] * rhs.y + q.adj[8] * rhs.z) * id);
            if (q.prism) {
                J[J_LA] = q.la0 + lam.x; J[J_LA + 1] = q.la1 + lam.y; J[J_LA + 2] = q.la2 + lam.z;
                imp_ang(A, B, lam);
            } else {
                J[J_LP] = q.lp.x + lam.x; J[J_LP + 1] = q.lp.y + lam.y; J[J_LP + 2] = q.lp.z + lam.z;
                imp_lin(A, B, q.rA, q.rB, lam);
            }
        }
    }
    {
        float Cd1, Cd2;
        if (q.prism) {
            V3 vr = relv(A, B, has_a, q.rA, q.rB);
            Cd1 = dot3(q.b1, vr); Cd2 = dot3(q.b2, vr);
        } else {
            V3 dw = B.w - A.w;
            Cd1 = dot3(q.b1, dw); Cd2 = dot3(q.b2, dw);
        }
        float r1 = Cd1 + brate * q.C1, r2 = Cd2 + brate * q.C2;
        if (q.det2 != 0.0f) {
            float id = 1.0f / q.det2;
            float l1 = -(q.k22 * r1 - q.k12 * r2) * id;
            float l2 = -(-q.k12 * r1 + q.k11 * r2) * id;
            if (q.prism) {
                J[J_LP] = q.lp.x + l1; J[J_LP + 1] = q.lp.y + l2;
                imp_lin(A, B, q.rA, q.rB, l1 * q.b1 + l2 * q.b2);
            } else {
                J[J_LA] = q.la0 + l1; J[J_LA + 1] = q.la1 + l2;
                imp_ang(A, B, l1 * q.b1 + l2 * q.b2);
            }
        }
    }
    if (q.kp != 0.0f || q.kd != 0.0f) {
        V3 ax = q.zA;
        float Cd = q.prism ? dot3(ax, relv(A, B, has_a, q.rA, q.rB)) : dot3(ax, B.w - A.w);
        float dl = -(Cd + q.bch + q.gam * q.ld) / q.kg;
        J[J_LD] = q.ld + dl;
        if (q.prism) imp_lin(A, B, q.rA, q.rB, dl * ax);
        else imp_ang(A, B, dl * ax);
    }
    if (q.lim) joint_limits(c, j, q.prism, A, B, has_a, q.rA, q.rB, q.zA, h, brate, false);
    store_body(c, q.a, A);
    store_body(c, q.b, B);
}

// ----------------------------------------------------------------------------- S1 AABB (exact)
// Half size along world axis r of a primitive with rotation rows R (add, multiply, abs only).
__device__ __forceinline__ float prim_half(int shape, float d0, float d1, float d2, float r0, float r1, float r2) {
    if (shape == 2) {
        float t0 = fabsf(r0) * d0;
        float t1 = fabsf(r1) * d1;
        float t2 = fabsf(r2) * d2;
        return (t0 + t1) + t2;
    }
    if (shape == 0) return d0;
    float t = fabsf(r2) * d1;
    return t + d0;
}
// A compound's box: along each world axis the largest |R c_k| + the part's own half size.
__device__ __forceinline__ void compound_half(const EnvCtx& c, int i, Qt q, const float R[3][3], float hm[3]) {
    const float* rec = comp_rec(c, i);
    const int np = gldi(reinterpret_cast<const int*>(rec));
    hm[0] = 0.0f; hm[1] = 0.0f; hm[2] = 0.0f;
    for (int k = 0; k < np; ++k) {
        const float4* P = reinterpret_cast<const float4*>(rec + 4 + 12 * k);
        const float4 r0 = gld4(P), r1 = gld4(P + 1), r2 = gld4(P + 2);
        const M3 Rk = rotm(qmul(q, Qt{r1.w, r2.x, r2.y, r2.z}));
        const int sh = __float_as_int(r0.x);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float o = R[r][0] * r1.x + R[r][1] * r1.y + R[r][2] * r1.z;
            const float hv = fabsf(o) + prim_half(sh, r0.y, r0.z, r0.w, Rk.m[r][0], Rk.m[r][1], Rk.m[r][2]);
            if (hv > hm[r]) hm[r] = hv;
        }
    }
}
template <bool COMP>
__device__ __forceinline__ void body_aabb(const EnvCtx& c, int i) {
#pragma clang fp contract(off)
    const Lay& l = c.lay;
    const int n = l.n;
    Qt q = ldp4(c, i, P_Q0);
    float xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    float xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    float wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    float R[3][3];
    R[0][0] = 1.0f - 2.0f * (yy + zz); R[0][1] = 2.0f * (xy - wz);        R[0][2] = 2.0f * (xz + wy);
    R[1][0] = 2.0f * (xy + wz);        R[1][1] = 1.0f - 2.0f * (xx + zz); R[1][2] = 2.0f * (yz - wx);
    R[2][0] = 2.0f * (xz - wy);        R[2][1] = 2.0f * (yz + wx);        R[2][2] = 1.0f - 2.0f * (xx + yy);
    int shape = iptr(c.L + l.SH)[i] & 0xFF;
    float d0 = c.L[l.DIM + i], d1 = c.L[l.DIM + n + i], d2 = c.L[l.DIM + 2 * n + i];
    float delta = c.bd->delta;
    float hm[3] = {0.0f, 0.0f, 0.0f};
    if (COMP && shape == SHAPE_COMPOUND) compound_half(c, i, q, R, hm);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float hv = (COMP && shape == SHAPE_COMPOUND) ? hm[r] : prim_half(shape, d0, d1, d2, R[r][0], R[r][1], R[r][2]);
        float half = hv + delta;
        float x = pose_rec(c, i)[P_X0 + r];
        c.L[l.AABB + r * n + i] = x - half;
        c.L[l.AABB + (3 + r) * n + i] = x + half;
    }
}

__device__ __forceinline__ bool aabb_overlap(const EnvCtx& c, int a, int b) {
    const float* A = c.L + c.lay.AABB;
    const int n = c.lay.n;
    for (int r = 0; r < 3; ++r)
        if (!(A[r * n + a] <= A[(3 + r) * n + b] && A[r * n + b] <= A[(3 + r) * n + a])) return false;
    return true;
}

// (pair_of lives in ms_dev.h)

// ----------------------------------------------------------------------------- schedule runner

// Walk a schedule: entry e = (start | count << 16) into the colour order; blocks of one entry
// touch disjoint dynamic bodies, so the lanes of the group run them concurrently.  `emax` is
// the wave-wide maximum number of entries (every lane reaches every barrier).
// Rows of one manifold block that stay fixed during a colour sweep (the block's own impulses
// change only in its own phase; body masses, inertias and pose offsets change only between
// sweeps).  A lane loads them for its next block at the end of the current phase, so a phase
// waits on one round of LDS loads (the two bodies' velocities) instead of a chain of them.
struct ManPre {
    int a, b, cnt;
    float ima, imb;
    S6 Ia, Ib;
    bool da, db;
    V3 rA[4], rB[4], n[4];
    float bias[4], mn[4], ln[4];
    V3 mrA, mrB, nb, t1;
    float mt1, mt2, mtw, mu, rt, lt1, lt2, ltw;
    int first;
};

template <bool SOLVE>
__device__ __forceinline__ void man_prefetch(const EnvCtx& c, int m, ManPre& p) {
    man_header(c, m, p.a, p.b, p.first, p.cnt);
    const int n = c.lay.n;
    p.da = is_dyn(c, p.a);
    p.db = is_dyn(c, p.b);
    p.ima = p.a >= 0 ? body_rec(c, p.a)[B_IM] : 0.0f;
    p.imb = body_rec(c, p.b)[B_IM];
    p.Ia = p.a >= 0 ? load_iw(c, p.a) : S6{0, 0, 0, 0, 0, 0};
    p.Ib = load_iw(c, p.b);
    (void)n;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < p.cnt) {
            const int q = p.first + k;
            p.rA[k] = pr3(c, R_RA, q);
            p.rB[k] = pr3(c, R_RB, q);
            p.n[k] = pr3(c, R_N, q);
            p.ln[k] = pr(c, R_LN, q);
            if (SOLVE) { p.bias[k] = pr(c, R_BIAS, q); p.mn[k] = pr(c, R_MN, q); }
        }
    }
    p.mrA = mf3(c, M_RA, m);
    p.mrB = mf3(c, M_RB, m);
    p.nb = mf3(c, M_NB, m);
    p.t1 = mf3(c, M_T1, m);
    p.lt1 = mf(c, M_LT1, m);
    p.lt2 = mf(c, M_LT2, m);
    p.ltw = mf(c, M_LTW, m);
    if (SOLVE) {
        p.mt1 = mf(c, M_MT1, m); p.mt2 = mf(c, M_MT2, m); p.mtw = mf(c, M_MTW, m);
        p.mu = mf(c, M_MU, m); p.rt = mf(c, M_RT, m);
    }
}

__device__ __forceinline__ void man_bodies(const EnvCtx& c, const ManPre& p, BodyR& A, BodyR& B) {
    const int n = c.lay.n;
    if (p.a >= 0) { A.v = ldv(c, p.a); A.w = ldw(c, p.a); }
    else { A.v = v3(0, 0, 0); A.w = v3(0, 0, 0); }
    B.v = ldv(c, p.b);
    B.w = ldw(c, p.b);
    A.im = p.ima; A.I = p.Ia; A.dyn = p.da;
    B.im = p.imb; B.I = p.Ib; B.dyn = p.db;
}

// One Gauss-Seidel visit of a manifold block: normal rows in point order (bias of the substep,
// clamped accumulated impulse), then the friction
// patch: two tangent rows and the twist row, clamped by mu and mu * r_t times the normal sum.
__device__ __forceinline__ void man_solve_pre(const EnvCtx& c, int m, const ManPre& p) {
    const bool has_a = p.a >= 0;
    BodyR A, B;
    man_bodies(c, p, A, B);
    float lsum = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < p.cnt) {
            const V3 rA = p.rA[k], rB = p.rB[k], n = p.n[k];
            float vn = dot3(relv(A, B, has_a, rA, rB), n);
            float dl = -p.mn[k] * (vn + p.bias[k]);
            float old = p.ln[k];
            float nl = fmaxf(old + dl, 0.0f);
            pr(c, R_LN, p.first + k) = nl;
            imp_lin(A, B, rA, rB, (nl - old) * n);
            lsum += nl;
        }
    }
    float lim = p.mu * lsum;
    V3 t2 = cross3(p.nb, p.t1);
    {
        float vt = dot3(relv(A, B, has_a, p.mrA, p.mrB), p.t1);
        float nl = fminf(fmaxf(p.lt1 - p.mt1 * vt, -lim), lim);
        mfr(c, M_LT1, m) = nl;
        imp_lin(A, B, p.mrA, p.mrB, (nl - p.lt1) * p.t1);
    }
    {
        float vt = dot3(relv(A, B, has_a, p.mrA, p.mrB), t2);
        float nl = fminf(fmaxf(p.lt2 - p.mt2 * vt, -lim), lim);
        mfr(c, M_LT2, m) = nl;
        imp_lin(A, B, p.mrA, p.mrB, (nl - p.lt2) * t2);
    }
    {
        float limw = p.rt * lim;
        float wr = dot3(p.nb, B.w - A.w);
        float nl = fminf(fmaxf(p.ltw - p.mtw * wr, -limw), limw);
        mfr(c, M_LTW, m) = nl;
        imp_ang(A, B, (nl - p.ltw) * p.nb);
    }
    store_body(c, p.a, A);
    store_body(c, p.b, B);
}

// ----------------------------------------------------------------------------- paired solve
// A manifold block visited by two lanes of a pair (lanes 2k, 2k + 1): the even lane holds body A,
// the odd lane body B.  Each lane forms its own body's velocity at its arm and gets the
// partner's over a cross-lane move; the relative velocity, the multiplier update and the clamps
// are then computed by both lanes alike, and each lane applies the impulse to its own body.
// Side A works with negated relative velocities and impulses: negation is exact and every
// product and sum here is symmetric under it, so both lanes see bit for bit the values of the
// one-lane visit (man_solve_pre), and A's update v + im (-P) equals v - im P.
__device__ __forceinline__ float pair_swap(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
}
__device__ __forceinline__ V3 pair_swap3(V3 v) { return v3(pair_swap(v.x), pair_swap(v.y), pair_swap(v.z)); }

struct ManHalf {
    int first, cnt;
    bool has, dyn;
    float im;
    S6 I;
    V3 r[4], n[4];
    float bias[4], mn[4], ln[4];
    V3 mr, nb, t1;
    float mt1, mt2, mtw, mu, rt, lt1, lt2, ltw;
    int body;
};

// Rows of manifold m for the lane holding side `sideB` (the arms of that side only).
__device__ __forceinline__ void man_prefetch_half(const EnvCtx& c, int m, bool sideB, ManHalf& p) {
    int a, b;
    man_header(c, m, a, b, p.first, p.cnt);
    p.body = sideB ? b : a;
    p.has = p.body >= 0;
    p.dyn = is_dyn(c, p.body);
    p.im = p.has ? body_rec(c, p.body)[B_IM] : 0.0f;
    p.I = p.has ? load_iw(c, p.body) : S6{0, 0, 0, 0, 0, 0};
    const int rrow = sideB ? R_RB : R_RA;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < p.cnt) {
            const int q = p.first + k;
            p.r[k] = pr3(c, rrow, q);
            p.n[k] = pr3(c, R_N, q);
            p.ln[k] = pr(c, R_LN, q);
            p.bias[k] = pr(c, R_BIAS, q);
            p.mn[k] = pr(c, R_MN, q);
        }
    }
    p.mr = mf3(c, sideB ? M_RB : M_RA, m);
    p.nb = mf3(c, M_NB, m);
    p.t1 = mf3(c, M_T1, m);
    p.lt1 = mf(c, M_LT1, m); p.lt2 = mf(c, M_LT2, m); p.ltw = mf(c, M_LTW, m);
    p.mt1 = mf(c, M_MT1, m); p.mt2 = mf(c, M_MT2, m); p.mtw = mf(c, M_MTW, m);
    p.mu = mf(c, M_MU, m); p.rt = mf(c, M_RT, m);
}

// The paired counterpart of man_solve_pre; both lanes of the pair must be active.
__device__ __forceinline__ void man_solve_half(const EnvCtx& c, int m, bool sideB, const ManHalf& p) {
    V3 v = p.has ? ldv(c, p.body) : v3(0, 0, 0);
    V3 w = p.has ? ldw(c, p.body) : v3(0, 0, 0);
    float lsum = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < p.cnt) {
            const V3 r = p.r[k], n = p.n[k];
            const V3 u = p.has ? v + cross3(w, r) : v3(0, 0, 0);
            const float d = dot3(u - pair_swap3(u), n);
            const float vn = sideB ? d : -d;
            const float dl = -p.mn[k] * (vn + p.bias[k]);
            const float old = p.ln[k];
            const float nl = fmaxf(old + dl, 0.0f);
            if (sideB) pr(c, R_LN, p.first + k) = nl;
            const V3 P = (sideB ? nl - old : -(nl - old)) * n;
            if (p.dyn) { v = v + p.im * P; w = w + muls(p.I, cross3(r, P)); }
            lsum += nl;
        }
    }
    const float lim = p.mu * lsum;
    const V3 t2 = cross3(p.nb, p.t1);
    {
        const V3 u = p.has ? v + cross3(w, p.mr) : v3(0, 0, 0);
        const float d = dot3(u - pair_swap3(u), p.t1);
        const float vt = sideB ? d : -d;
        const float nl = fminf(fmaxf(p.lt1 - p.mt1 * vt, -lim), lim);
        if (sideB) mfr(c, M_LT1, m) = nl;
        const V3 P = (sideB ? nl - p.lt1 : -(nl - p.lt1)) * p.t1;
        if (p.dyn) { v = v + p.im * P; w = w + muls(p.I, cross3(p.mr, P)); }
    }
    {
        const V3 u = p.has ? v + cross3(w, p.mr) : v3(0, 0, 0);
        const float d = dot3(u - pair_swap3(u), t2);
        const float vt = sideB ? d : -d;
        const float nl = fminf(fmaxf(p.lt2 - p.mt2 * vt, -lim), lim);
        if (sideB) mfr(c, M_LT2, m) = nl;
        const V3 P = (sideB ? nl - p.lt2 : -(nl - p.lt2)) * t2;
        if (p.dyn) { v = v + p.im * P; w = w + muls(p.I, cross3(p.mr, P)); }
    }
    {
        const float limw = p.rt * lim;
        const float d = dot3(p.nb, w - pair_swap3(w));
        const float wr = sideB ? d : -d;
        const float nl = fminf(fmaxf(p.ltw - p.mtw * wr, -limw), limw);
        if (sideB) mfr(c, M_LTW, m) = nl;
        const V3 L = (sideB ? nl - p.ltw : -(nl - p.ltw)) * p.nb;
        if (p.dyn) w = w + muls(p.I, L);
    }
    if (p.dyn) { stv(c, p.body, v); stw(c, p.body, w); }
}

// Bias of every contact point for the sweeps of one substep.  The pose offsets change only
// when a substep integrates, so the current separation s = s0 + n . (dB - dA) of each point (the
// displacement of its body-fixed arms since the step start) and its bias (speculative s / h for
// a gap; Baumgarte beta s / h capped at the maximum depenetration velocity for a penetration, or
// none in a velocity pass) are the same in every colour of the substep: one pass, a lane per
// manifold, computes them before the sweeps.
__device__ __forceinline__ void bias_pass(const EnvCtx& c, int nman, float h, bool vpass, int li, int G) {
    const BatchDev& bd = *c.bd;
    for (int m = li; m < nman; m += G) {
        int a, b, first, cnt;
        man_header(c, m, a, b, first, cnt);
        const bool has_a = a >= 0;
        const PoseR pa = load_pose(c, a), pb = load_pose(c, b);
        // the rows of all four slots are read before any arithmetic (one LDS round trip); the
        // rows past the block's count lie inside the env's region and are not used
        V3 rA[4], rB[4], nq[4];
        float s0[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = first + k;
            rA[k] = pr3(c, R_RA, q); rB[k] = pr3(c, R_RB, q); nq[k] = pr3(c, R_N, q); s0[k] = pr(c, R_S0, q);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < cnt) {
                V3 dA = has_a ? disp(pa, rA[k]) : v3(0, 0, 0);
                V3 dB = disp(pb, rB[k]);
                float s = s0[k] + dot3(nq[k], dB - dA);
                float bias;
                if (s > 0.0f) bias = s / h;
                else bias = vpass ? 0.0f : fmaxf(bd.beta * s / h, -bd.max_depen);
                pr(c, R_BIAS, first + k) = bias;
            }
        }
    }
}

// Per-body block lists for the warm start: for every dynamic body, the blocks (joints, then
// manifolds, numbered as in the schedule) touching it in colour order with the body's side.  A
// body sits in at most one block per colour, and a warm-start impulse does not depend on any
// velocity, so applying a body's blocks in this order reproduces, bit for bit, what a coloured
// warm sweep (every block of a colour applying its impulses to both bodies) does to that body.
// Built once per step (after colouring) in the candidate area: offsets [n + 1] ints, then u16
// entries (block | side << 15).
// nn: the env's body count, 0 for a frozen env or an empty slot of the tile (which must not
// touch the LDS it aliases).
__device__ __forceinline__ void block_bodies(const EnvCtx& c, int blk, int& a, int& b) {
    if (blk < c.lay.nj) {
        const int* J = reinterpret_cast<const int*>(jrec(c, blk));
        a = J[J_PA];
        b = J[J_CH];
    } else {
        int f, cnt;
        man_header(c, blk - c.lay.nj, a, b, f, cnt);
    }
}
__device__ __forceinline__ void build_body_lists(const EnvCtx& c, int nn, int nman, int li, int G) {
    const Lay& l = c.lay;
    const int n = nn;
    const int nb = l.nj + nman;   // blocks: joints, then manifolds
    int* OFF = iptr(c.L + l.CAND);
    uint16_t* ENT = reinterpret_cast<uint16_t*>(OFF + l.n + 1);
    const uint16_t* ORD = reinterpret_cast<const uint16_t*>(c.L + l.ORDER);
    // degree of every body: lane per body, blocks in colour order
    for (int i = li; i < n; i += G) {
        int deg = 0;
        if (is_dyn(c, i)) {
            for (int p = 0; p < nb; ++p) {
                int a, b;
                block_bodies(c, int(ORD[p]), a, b);
                deg += (a == i ? 1 : 0) + (b == i ? 1 : 0);
            }
        }
        OFF[i + 1] = deg;
    }
    wave_sync();
    if (li == 0 && n > 0) {
        OFF[0] = 0;
        for (int i = 0; i < n; ++i) OFF[i + 1] += OFF[i];
    }
    wave_sync();
    for (int i = li; i < n; i += G) {
        if (!is_dyn(c, i)) continue;
        int o = OFF[i];
        for (int p = 0; p < nb; ++p) {
            const int blk = int(ORD[p]);
            int a, b;
            block_bodies(c, blk, a, b);
            if (a == i) ENT[o++] = uint16_t(blk);
            if (b == i) ENT[o++] = uint16_t(blk | 0x8000);
        }
    }
}

// The same lists for a wavefront holding one env (G = 64): the headers of the blocks in colour
// order sit in registers (lane p holds position p, p + 64, p + 128), and every body lane walks
// them with scalar reads of those registers instead of a chain of dependent LDS loads.
__device__ __forceinline__ void build_body_lists_wave(const EnvCtx& c, int nn, int nman_in, int li) {
    const Lay& l = c.lay;
    const int n = __builtin_amdgcn_readfirstlane(nn);
    const int nman = __builtin_amdgcn_readfirstlane(l.nj + nman_in);   // blocks: joints, then manifolds
    int* OFF = iptr(c.L + l.CAND);
    uint16_t* ENT = reinterpret_cast<uint16_t*>(OFF + l.n + 1);
    const uint16_t* ORD = reinterpret_cast<const uint16_t*>(c.L + l.ORDER);
    // (block << 16) | a | b << 8 of colour position r * 64 + li (a = 0xFF for the world or the
    // ground); 0xFFFF never matches a body
    int hd[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int p = r * WAVE + li;
        int w = 0xFFFF;
        if (p < nman) {
            const int blk = int(ORD[p]);
            int a, b;
            block_bodies(c, blk, a, b);
            w = (a < 0 ? 0xFF : a) | (b << 8) | (blk << 16);
        }
        hd[r] = w;
    }
    const bool mine = li < n && is_dyn(c, li);
    int deg = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int kend = min(WAVE, nman - r * WAVE);
        for (int k = 0; k < kend; ++k) {
            const int w = __builtin_amdgcn_readlane(hd[r], k);
            deg += ((w & 0xFF) == li ? 1 : 0) + (((w >> 8) & 0xFF) == li ? 1 : 0);
        }
    }
    if (!mine) deg = 0;
    // exclusive prefix of the degrees over the body lanes
    int incl = deg;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (li >= d) incl += y;
    }
    if (li < n) OFF[li + 1] = incl;
    if (li == 0 && n > 0) OFF[0] = 0;
    int o = incl - deg;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int kend = min(WAVE, nman - r * WAVE);
        for (int k = 0; k < kend; ++k) {
            const int w = __builtin_amdgcn_readlane(hd[r], k);
            const int m = w >> 16;
            if (mine && (w & 0xFF) == li) ENT[o++] = uint16_t(m);
            if (mine && ((w >> 8) & 0xFF) == li) ENT[o++] = uint16_t(m | 0x8000);
        }
    }
}

// Warm-start impulses of manifold m (points first .. first + cnt - 1) applied to one of its bodies
// (side B adds, side A subtracts), as the coloured warm sweep applies them to that body.
__device__ __forceinline__ void warm_manifold(const EnvCtx& c, int m, int first, int cnt, bool sideB, float im,
                                              const S6& I, V3& v, V3& w) {
    const int rrow = sideB ? R_RB : R_RA;
    const int mrow = sideB ? M_RB : M_RA;
    // every row of the block is read before any arithmetic (one LDS round trip); the
    // rows past the block's count lie inside the env's region and are not used
    float ln[4];
    V3 nq[4], rq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int q = first + k;
        ln[k] = pr(c, R_LN, q);
        nq[k] = pr3(c, R_N, q);
        rq[k] = pr3(c, rrow, q);
    }
    const V3 t1 = mf3(c, M_T1, m), nb = mf3(c, M_NB, m), mr = mf3(c, mrow, m);
    const float lt1 = mf(c, M_LT1, m), lt2 = mf(c, M_LT2, m), ltw = mf(c, M_LTW, m);
    // side A receives the negated impulses; negating the multiplier negates every product
    // and sum below exactly, so adding them equals subtracting the unnegated ones
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < cnt) {
            const V3 P = (sideB ? ln[k] : -ln[k]) * nq[k];
            v = v + im * P;
            w = w + muls(I, cross3(rq[k], P));
        }
    }
    const V3 t2 = cross3(nb, t1);
    const V3 P = (sideB ? lt1 : -lt1) * t1 + (sideB ? lt2 : -lt2) * t2;
    const V3 L = (sideB ? ltw : -ltw) * nb;
    v = v + im * P;
    w = w + muls(I, cross3(mr, P));
    w = w + muls(I, L);
}

// Gravity and damping of one dynamic body for a substep, then (after the first substep) its
// warm start: the accumulated impulses of its blocks in colour order, as imp_lin / imp_ang apply
// them to this body (side A subtracts, side B adds).
__device__ __forceinline__ void body_substep_start(const EnvCtx& c, int i, float h, float ldmp, float admp, bool warm) {
    const BatchDev& bd = *c.bd;
    const Lay& l = c.lay;
    const int n = l.n;
    V3 v = ldv(c, i);
    v = ldmp * (v + h * v3(bd.gx, bd.gy, bd.gz));
    V3 w = admp * ldw(c, i);
    if (warm) {
        const float im = body_rec(c, i)[B_IM];
        const S6 I = load_iw(c, i);
        const int* OFF = iptr(c.L + l.CAND);
        const uint16_t* ENT = reinterpret_cast<const uint16_t*>(OFF + n + 1);
        // the next block's entry and header are read while this block's rows are in use
        const int e0 = OFF[i], e1 = OFF[i + 1];
        int ent = e0 < e1 ? ENT[e0] : 0;   // manifold 0 always exists: the header read stays in range
        int fc = iptr(c.L + l.MAN + (ent & 0x7FFF) * M_WORDS)[M_FC];
        for (int e = e0; e < e1; ++e) {
            const int m = ent & 0x7FFF;
            const bool sideB = (ent >> 15) != 0;
            const int first = fc & 0xFFFF, cnt = fc >> 16;
            const int ent_next = ENT[e + 1 < e1 ? e + 1 : e];
            const int fc_next = iptr(c.L + l.MAN + (ent_next & 0x7FFF) * M_WORDS)[M_FC];
            warm_manifold(c, m, first, cnt, sideB, im, I, v, w);
            ent = ent_next;
            fc = fc_next;
        }
    }
    stv(c, i, v);
    stw(c, i, w);
}

// Warm start of one dynamic body of a wavefront with joints, after the substep's joint pass: the
// accumulated impulses of its blocks in colour order: a joint's point impulse at its arm, its
// two angular-block impulses about the frame axes and its drive impulse about the joint axis; a
// manifold's as warm_manifold (side A with negated multipliers, which is exact).
__device__ __forceinline__ void body_warm_gather(const EnvCtx& c, int i) {
    const Lay& l = c.lay;
    V3 v = ldv(c, i), w = ldw(c, i);
    const float im = body_rec(c, i)[B_IM];
    const S6 I = load_iw(c, i);
    const int* OFF = iptr(c.L + l.CAND);
    const uint16_t* ENT = reinterpret_cast<const uint16_t*>(OFF + l.n + 1);
    for (int e = OFF[i]; e < OFF[i + 1]; ++e) {
        const int ent = ENT[e];
        const int blk = ent & 0x7FFF;
        const bool sideB = (ent >> 15) != 0;
        if (blk < l.nj) {
            const float* P = jinv(c, blk);
            const float* J = jrec(c, blk);
            const V3 r = jv3(P, sideB ? JI_RB : JI_RA), zA = jv3(P, JI_ZA), b1 = jv3(P, JI_B1), b2 = jv3(P, JI_B2);
            const float ld = sideB ? J[J_LD] : -J[J_LD];
            const float lim = sideB ? J[J_LL] - J[J_LL + 1] : -(J[J_LL] - J[J_LL + 1]);
            if (!jprism(J)) {
                // point impulse at the arm, the angular block about b1, b2, drive and limits about zA
                const V3 lp = sideB ? v3(J[J_LP], J[J_LP + 1], J[J_LP + 2]) : v3(-J[J_LP], -J[J_LP + 1], -J[J_LP + 2]);
                const float la0 = sideB ? J[J_LA] : -J[J_LA], la1 = sideB ? J[J_LA + 1] : -J[J_LA + 1];
                v = v + im * lp;
                w = w + muls(I, cross3(r, lp));
                w = w + muls(I, la0 * b1 + la1 * b2);
                w = w + muls(I, ld * zA);
                if (jlimited(J)) w = w + muls(I, lim * zA);
            } else {
                // rows across the slide axis at the arm, the rotation lock, drive and limits along zA
                const float p0 = sideB ? J[J_LP] : -J[J_LP], p1 = sideB ? J[J_LP + 1] : -J[J_LP + 1];
                const V3 la = sideB ? v3(J[J_LA], J[J_LA + 1], J[J_LA + 2]) : v3(-J[J_LA], -J[J_LA + 1], -J[J_LA + 2]);
                const V3 P1 = p0 * b1 + p1 * b2;
                v = v + im * P1;
                w = w + muls(I, cross3(r, P1));
                w = w + muls(I, la);
                const V3 P2 = ld * zA;
                v = v + im * P2;
                w = w + muls(I, cross3(r, P2));
                if (jlimited(J)) {
                    const V3 P3 = lim * zA;
                    v = v + im * P3;
                    w = w + muls(I, cross3(r, P3));
                }
            }
        } else {
            const int m = blk - l.nj;
            int a, b, first, cnt;
            man_header(c, m, a, b, first, cnt);
            warm_manifold(c, m, first, cnt, sideB, im, I, v, w);
        }
    }
    stv(c, i, v);
    stw(c, i, w);
}

enum { OP_SOLVE = 1, OP_VSOLVE = 2, OP_REST = 3, OP_JOINT = 4 };

// Block of this lane at schedule entry e (-1: none).
__device__ __forceinline__ int sched_block(const EnvCtx& c, int sched_off, int nsched, int e, int li) {
    if (e >= nsched) return -1;
    const int ent = reinterpret_cast<const int*>(c.L + sched_off)[e];
    const int start = ent & 0xFFFF, cnt = ent >> 16;
    if (li >= cnt) return -1;
    return reinterpret_cast<const uint16_t*>(c.L + c.lay.ORDER)[start + li];
}

// One sweep over a schedule: entry by entry (colour order), each lane visiting its block of the
// entry, a wavefront sync between entries.  A manifold block of a solve sweep runs from its rows
// loaded in one batch; when no env of the wave has joints (PIPE) the rows of a lane's
// next block are loaded at the end of the current entry, behind the compute of this one.
template <int OP, bool PIPE>
__device__ __forceinline__ void run_schedule(const EnvCtx& c, int sched_off, int nsched, int emax, float h, int li) {
    const Lay& l = c.lay;
    if (OP == OP_JOINT) {   // joint-only schedule: every block is a joint
        const float brate = c.bd->beta_j / c.bd->dt;
        int blk = sched_block(c, sched_off, nsched, 0, li);
        JointPre jp;
        if (blk >= 0) joint_prefetch(c, blk, jp);
        for (int e = 0; e < emax; ++e) {
            if (blk >= 0) joint_solve_pre(c, blk, jp, brate, h);
            blk = sched_block(c, sched_off, nsched, e + 1, li);
            if (blk >= 0) joint_prefetch(c, blk, jp);
            wave_sync();
        }
        return;
    }
    constexpr bool PRE = OP == OP_SOLVE || OP == OP_VSOLVE;
    constexpr bool SOLVE = OP == OP_SOLVE || OP == OP_VSOLVE;
    int blk = sched_block(c, sched_off, nsched, 0, li);
    ManPre pre;
    if (PIPE && PRE && blk >= 0) man_prefetch<SOLVE>(c, blk - l.nj, pre);
    for (int e = 0; e < emax; ++e) {
        if (blk >= 0) {
            if (!PIPE && blk < l.nj) {
                if (OP == OP_SOLVE || OP == OP_JOINT) joint_solve(c, blk, h, false);
                else if (OP == OP_VSOLVE) joint_solve(c, blk, h, true);
            } else {
                const int m = blk - l.nj;
                if (!PIPE && PRE) man_prefetch<SOLVE>(c, m, pre);
                if (OP == OP_SOLVE || OP == OP_VSOLVE) man_solve_pre(c, m, pre);
                else if (OP == OP_REST) manifold_restitution(c, m);
            }
        }
        blk = sched_block(c, sched_off, nsched, e + 1, li);
        if (PIPE && PRE && blk >= 0) man_prefetch<SOLVE>(c, blk - l.nj, pre);
        wave_sync();
    }
}

// The solve sweep of a joint-free env with paired lanes: lane pair k (lanes 2k, 2k + 1 of the
// group) visits blocks k, k + G / 2, ... of each entry (the blocks of one colour share no dynamic
// body, so any split of a colour is the same sweep), the rows of its next block loaded behind
// the compute of the current one.
__device__ __forceinline__ void run_schedule_pairs(const EnvCtx& c, int sched_off, int nsched, int emax, int li, int G) {
    const Lay& l = c.lay;
    const int hg = G >> 1, slot = li >> 1;
    const bool sideB = (li & 1) != 0;
    const uint16_t* ORD = reinterpret_cast<const uint16_t*>(c.L + l.ORDER);
    const int* SCH = reinterpret_cast<const int*>(c.L + sched_off);
    int ent = nsched > 0 ? SCH[0] : 0;
    int idx = slot;
    int blk = idx < (ent >> 16) ? int(ORD[(ent & 0xFFFF) + idx]) : -1;
    ManHalf pre;
    if (blk >= 0) man_prefetch_half(c, blk - l.nj, sideB, pre);
    for (int e = 0; e < emax; ++e) {
        while (blk >= 0) {
            man_solve_half(c, blk - l.nj, sideB, pre);
            idx += hg;
            blk = idx < (ent >> 16) ? int(ORD[(ent & 0xFFFF) + idx]) : -1;
            if (blk >= 0) man_prefetch_half(c, blk - l.nj, sideB, pre);
        }
        ent = e + 1 < nsched ? SCH[e + 1] : 0;
        idx = slot;
        blk = idx < (ent >> 16) ? int(ORD[(ent & 0xFFFF) + idx]) : -1;
        if (blk >= 0) man_prefetch_half(c, blk - l.nj, sideB, pre);
        wave_sync();
    }
}

// ----------------------------------------------------------------------------- S5 colouring
// Serial greedy colouring by the group leader: blocks = joints (index order) then manifolds
// (canonical order); each block takes the smallest colour unused by its dynamic bodies.  Then a
// stable counting sort by colour and the two schedules (all blocks; joints only).
__device__ __forceinline__ void colour_env(const EnvCtx& c, int G) {
    const Lay& l = c.lay;
    int* SC = iptr(c.L + l.SCAL);
    const int nman = SC[SC_NMAN];
    const int nb = l.nj + nman;
    uint16_t* BC = reinterpret_cast<uint16_t*>(c.L + l.BCOL);
    uint16_t* ORD = reinterpret_cast<uint16_t*>(c.L + l.ORDER);
    int* CS = iptr(c.L + l.CSTART);
    int* CMi = iptr(c.L + l.CM);
    for (int k = 0; k <= N_COLOURS + 1; ++k) CS[k] = 0;
    int ncol = 0;
    bool overflow = false;
    for (int blk = 0; blk < nb; ++blk) {
        int a, b;
        if (blk < l.nj) {
            const int* J = reinterpret_cast<const int*>(jrec(c, blk));
            a = J[J_PA]; b = J[J_CH];
        } else {
            int f, cnt;
            man_header(c, blk - l.nj, a, b, f, cnt);
        }
        bool da = is_dyn(c, a), db = is_dyn(c, b);
        uint64_t u = 0;
        if (da) u |= uint64_t(uint32_t(CMi[2 * a])) | (uint64_t(uint32_t(CMi[2 * a + 1])) << 32);
        if (db) u |= uint64_t(uint32_t(CMi[2 * b])) | (uint64_t(uint32_t(CMi[2 * b + 1])) << 32);
        int col;
        if (~u == 0) { col = N_COLOURS; overflow = true; }
        else {
            col = __ffsll((unsigned long long)(~u)) - 1;
            uint64_t bit = uint64_t(1) << col;
            if (da) { uint64_t m = (uint64_t(uint32_t(CMi[2 * a])) | (uint64_t(uint32_t(CMi[2 * a + 1])) << 32)) | bit;
                      CMi[2 * a] = int(uint32_t(m)); CMi[2 * a + 1] = int(uint32_t(m >> 32)); }
            if (db) { uint64_t m = (uint64_t(uint32_t(CMi[2 * b])) | (uint64_t(uint32_t(CMi[2 * b + 1])) << 32)) | bit;
                      CMi[2 * b] = int(uint32_t(m)); CMi[2 * b + 1] = int(uint32_t(m >> 32)); }
        }
        BC[blk] = uint16_t(col);
        CS[col + 1] += 1;
        if (col + 1 > ncol) ncol = col + 1;
    }
    if (overflow) SC[SC_STATUS] |= 4;
    for (int k = 0; k <= N_COLOURS; ++k) CS[k + 1] += CS[k];
    // stable scatter, using the joint schedule area as per-colour cursors
    int* cur = iptr(c.L + l.JSCHED);
    for (int k = 0; k <= N_COLOURS; ++k) cur[k] = CS[k];
    for (int blk = 0; blk < nb; ++blk) ORD[cur[BC[blk]]++] = uint16_t(blk);
    int* SCH = iptr(c.L + l.SCHED);
    int ns = 0;
    for (int col = 0; col < ncol; ++col) {
        int s0 = CS[col], cnt = CS[col + 1] - s0;
        if (col < N_COLOURS) {
            for (int o = 0; o < cnt; o += G) SCH[ns++] = (s0 + o) | (min(G, cnt - o) << 16);
        } else {
            for (int o = 0; o < cnt; ++o) SCH[ns++] = (s0 + o) | (1 << 16);
        }
    }
    int* JS = iptr(c.L + l.JSCHED);
    int njs = 0;
    if (l.nj > 0) {
        for (int col = 0; col < ncol; ++col) {
            int s0 = CS[col], cnt = 0;
            while (s0 + cnt < CS[col + 1] && ORD[s0 + cnt] < l.nj) ++cnt;
            if (col < N_COLOURS) {
                for (int o = 0; o < cnt; o += G) JS[njs++] = (s0 + o) | (min(G, cnt - o) << 16);
            } else {
                for (int o = 0; o < cnt; ++o) JS[njs++] = (s0 + o) | (1 << 16);
            }
        }
    }
    SC[SC_NCOL] = ncol;
    SC[SC_NSCHED] = ns;
    SC[SC_NJSCHED] = njs;
}

// The same greedy colouring and stable sort for an env that owns the whole wave (64 lanes): the
// colour masks of the bodies live in registers (body i in lane i) and the greedy loop runs on
// uniform values read across lanes, so a block costs a few scalar instructions instead of a
// chain of LDS round trips.  Block order, colours and schedules equal those of colour_env.
__device__ __forceinline__ void colour_env_wave(const EnvCtx& c) {
    const Lay& l = c.lay;
    const int li = int(threadIdx.x) & (WAVE - 1);
    int* SC = iptr(c.L + l.SCAL);
    // one env per wave: its sizes are wave-uniform (scalar loop bounds)
    const int nj = __builtin_amdgcn_readfirstlane(l.nj);
    const int nman = __builtin_amdgcn_readfirstlane(SC[SC_NMAN]);
    const int nb = nj + nman;
    uint16_t* BC = reinterpret_cast<uint16_t*>(c.L + l.BCOL);
    uint16_t* ORD = reinterpret_cast<uint16_t*>(c.L + l.ORDER);
    const uint64_t dynm = __ballot(li < l.n && is_dyn(c, li));
    uint32_t mlo = 0, mhi = 0;   // colours used by body li
    int ccnt = 0, jcnt = 0;      // blocks / joint blocks of colour li
    int c64 = 0, j64 = 0;        // the same for the overflow colour
    int ncol = 0;
    bool overflow = false;
    for (int r = 0; r * WAVE < nb; ++r) {
        const int blk = r * WAVE + li;
        int pk = 0xFFFFFFFF;
        if (blk < nb) {
            int a, b;
            if (blk < nj) {
                const int* J = reinterpret_cast<const int*>(jrec(c, blk));
                a = J[J_PA]; b = J[J_CH];
            } else {
                int f, cnt;
                man_header(c, blk - nj, a, b, f, cnt);
            }
            pk = (a & 0xFFFF) | (b << 16);
        }
        const int kend = min(WAVE, nb - r * WAVE);
        int mycol = 0;
        for (int k = 0; k < kend; ++k) {
            const int w = __builtin_amdgcn_readlane(pk, k);
            const int a = int(int16_t(w & 0xFFFF)), b = w >> 16;
            const bool da = a >= 0 && ((dynm >> a) & 1), db = b >= 0 && ((dynm >> b) & 1);
            uint64_t u = 0;
            if (da) u |= uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mlo), a))) |
                         (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mhi), a))) << 32);
            if (db) u |= uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mlo), b))) |
                         (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(mhi), b))) << 32);
            int col;
            const bool joint = r * WAVE + k < nj;
            if (~u == 0) {
                col = N_COLOURS;
                overflow = true;
                c64 += 1;
                j64 += joint ? 1 : 0;
            } else {
                col = __ffsll((unsigned long long)(~u)) - 1;
                const uint32_t blo = col < 32 ? (1u << col) : 0u, bhi = col < 32 ? 0u : (1u << (col - 32));
                if ((da && li == a) || (db && li == b)) { mlo |= blo; mhi |= bhi; }
                if (li == col) { ccnt += 1; jcnt += joint ? 1 : 0; }
            }
            if (li == k) mycol = col;
            ncol = max(ncol, col + 1);
        }
        if (blk < nb) BC[blk] = uint16_t(mycol);
    }
    if (overflow && li == 0) SC[SC_STATUS] |= 4;
    // colour starts: inclusive prefix of the per-colour counts over the lanes
    int incl = ccnt;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(incl, d);
        if (li >= d) incl += y;
    }
    const int start = incl - ccnt;                         // first slot of colour li
    const int start64 = __builtin_amdgcn_readlane(incl, WAVE - 1);
    // stable scatter by colour: rank = earlier blocks of the same colour
    int seen = 0;      // blocks of colour li placed so far
    int seen64 = 0;
    for (int r = 0; r * WAVE < nb; ++r) {
        const int blk = r * WAVE + li;
        const bool valid = blk < nb;
        const int col = valid ? int(BC[blk]) : -1;
        for (int k = 0; k < ncol; ++k) {
            const uint64_t m = __ballot(col == k);
            if (m == 0) continue;
            const int base = k < N_COLOURS ? __builtin_amdgcn_readlane(start, k) + __builtin_amdgcn_readlane(seen, k)
                                           : start64 + seen64;
            if (col == k) ORD[base + __popcll(m & ((uint64_t(1) << li) - 1))] = uint16_t(blk);
            if (k < N_COLOURS) { if (li == k) seen += __popcll(m); }
            else seen64 += __popcll(m);
        }
    }
    // schedules: entries of <= 64 blocks per parallel colour, one entry per overflow block
    if (li == 0) {
        int* SCH = iptr(c.L + l.SCHED);
        int* JS = iptr(c.L + l.JSCHED);
        int ns = 0, njs = 0;
        for (int col = 0; col < ncol; ++col) {
            const int s0 = col < N_COLOURS ? __builtin_amdgcn_readlane(start, col) : start64;
            const int cnt = col < N_COLOURS ? __builtin_amdgcn_readlane(ccnt, col) : c64;
            const int jc = col < N_COLOURS ? __builtin_amdgcn_readlane(jcnt, col) : j64;
            if (col < N_COLOURS) {
                for (int o = 0; o < cnt; o += WAVE) SCH[ns++] = (s0 + o) | (min(WAVE, cnt - o) << 16);
                for (int o = 0; o < jc; o += WAVE) JS[njs++] = (s0 + o) | (min(WAVE, jc - o) << 16);
            } else {
                for (int o = 0; o < cnt; ++o) SCH[ns++] = (s0 + o) | (1 << 16);
                for (int o = 0; o < jc; ++o) JS[njs++] = (s0 + o) | (1 << 16);
            }
        }
        SC[SC_NCOL] = ncol;
        SC[SC_NSCHED] = ns;
        SC[SC_NJSCHED] = nj > 0 ? njs : 0;
    }
}

// S3 for one candidate: decode the pair, run the narrowphase in a frame centred on body A (or
// on the ground below the body) and reduce to <= 4 points; code < 0 means no candidate.
__device__ __forceinline__ void np_candidate(const EnvCtx& c, int code, NOut& o, int& a, int& b, bool& plane, V3& base,
                                          V3& offB) {
    o.mask = 0;
    o.decision = 0;
    base = v3(0, 0, 0);
    offB = v3(0, 0, 0);
    if (code < 0) return;
    const Lay& l = c.lay;
    const BatchDev& bd = *c.bd;
    const int n = l.n;
    a = code & 0xFF;
    b = code >> 8;
    plane = b == n;
    {
        int* SC = iptr(c.L + l.SCAL);
        int sa = iptr(c.L + l.SH)[a] & 0xFF;
        int kind;
        if (plane) kind = 9 + sa;
        else {
            int sb2 = iptr(c.L + l.SH)[b] & 0xFF;
            kind = 3 * min(sa, sb2) + max(sa, sb2);
        }
        atomicAdd(&SC[16 + STAT_KIND0 + kind], 1);
    }
    V3 xa = ldp3(c, a, P_X0);
    if (plane) {
        Shp sb = shape_of(c, a, v3(0.0f, 0.0f, xa.z - bd.plane_z));
        base = v3(xa.x, xa.y, bd.plane_z);
        offB = sb.c;
        np_plane(o, sb, bd.delta);
    } else {
        Shp sa = shape_of(c, a, v3(0, 0, 0));
        Shp sb = shape_of(c, b, ldp3(c, b, P_X0) - xa);
        base = xa;
        offB = sb.c;
        np_pair(o, sa, sb, bd.delta);
    }
    reduce4(o);
    compact4(o);
}

// S4 for one kept pair: a normal row per kept point (arms from the step-start centres, pre-step
// normal velocity, effective mass) and the manifold's friction patch at the points' centroid.
__device__ __forceinline__ void write_rows(const EnvCtx& c, const NOut& o, int k, int a, int b, bool plane, V3 base,
                                        V3 offB, int keep, int first, int m, int part, bool dbg, int dpo, int dmo) {
    const Lay& l = c.lay;
    const BatchDev& bd = *c.bd;
    int ia = plane ? -1 : a, ib = plane ? a : b;
    float mu, e;
    if (plane) { mu = (bd.plane_mu + c.L[l.MU + a]) / 2.0f; e = fmaxf(bd.plane_e, c.L[l.EE + a]); }
    else { mu = (c.L[l.MU + a] + c.L[l.MU + b]) / 2.0f; e = fmaxf(c.L[l.EE + a], c.L[l.EE + b]); }
    V3 csum = v3(0, 0, 0), nsum = v3(0, 0, 0);
#pragma unroll
    for (int K = 0; K < 4; ++K) {
        if (K >= keep) continue;   // the kept points are slots 0 .. keep - 1
        int kk = first + K;
        V3 p = o.pt[K].p, nv = o.pt[K].n;
        V3 rA = ia >= 0 ? p : v3(0, 0, 0);
        V3 rB = p - offB;
        V3 vrel = rel_vel(c, ia, ib, rA, rB);
        pr(c, R_RA, kk) = rA.x; pr(c, R_RA + 1, kk) = rA.y; pr(c, R_RA + 2, kk) = rA.z;
        pr(c, R_RB, kk) = rB.x; pr(c, R_RB + 1, kk) = rB.y; pr(c, R_RB + 2, kk) = rB.z;
        pr(c, R_N, kk) = nv.x; pr(c, R_N + 1, kk) = nv.y; pr(c, R_N + 2, kk) = nv.z;
        pr(c, R_MN, kk) = eff_mass(c, ia, ib, rA, rB, nv);
        pr(c, R_S0, kk) = o.pt[K].s;
        pr(c, R_VN, kk) = dot3(vrel, nv);
        pr(c, R_LN, kk) = 0.0f;
        csum = csum + p;
        nsum = nsum + nv;
        if (dbg) {
            float* dq = bd.dbg_pts + 8 * size_t(dpo + kk);
            V3 pw = base + p;
            dq[0] = pw.x; dq[1] = pw.y; dq[2] = pw.z; dq[3] = nv.x; dq[4] = nv.y; dq[5] = nv.z;
            dq[6] = o.pt[K].s; dq[7] = 0.0f;
        }
    }
    V3 cc = (1.0f / float(keep)) * csum;
    V3 nb = (1.0f / len3(nsum)) * nsum;
    V3 rA = ia >= 0 ? cc : v3(0, 0, 0);
    V3 rB = cc - offB;
    V3 vrel = rel_vel(c, ia, ib, rA, rB);
    V3 vt = vrel - dot3(vrel, nb) * nb;
    float vtl = len3(vt);
    V3 t1 = vtl >= 1e-3f ? (1.0f / vtl) * vt : onb_t1(nb);
    V3 t2 = cross3(nb, t1);
    float kw = (ia >= 0 ? dot3(nb, muls(load_iw(c, ia), nb)) : 0.0f) + dot3(nb, muls(load_iw(c, ib), nb));
    float rsum = 0.0f;
#pragma unroll
    for (int K = 0; K < 4; ++K)
        if (K < keep) rsum += len3(o.pt[K].p - cc);
    iptr(c.L + l.MAN + m * M_WORDS)[M_AB] = (ia < 0 ? 0xFF : ia) | (ib << 8) | (part << 16);
    iptr(c.L + l.MAN + m * M_WORDS)[M_FC] = first | (keep << 16);
    mfr(c, M_RA, m) = rA.x; mfr(c, M_RA + 1, m) = rA.y; mfr(c, M_RA + 2, m) = rA.z;
    mfr(c, M_RB, m) = rB.x; mfr(c, M_RB + 1, m) = rB.y; mfr(c, M_RB + 2, m) = rB.z;
    mfr(c, M_NB, m) = nb.x; mfr(c, M_NB + 1, m) = nb.y; mfr(c, M_NB + 2, m) = nb.z;
    mfr(c, M_T1, m) = t1.x; mfr(c, M_T1 + 1, m) = t1.y; mfr(c, M_T1 + 2, m) = t1.z;
    mfr(c, M_MT1, m) = eff_mass(c, ia, ib, rA, rB, t1);
    mfr(c, M_MT2, m) = eff_mass(c, ia, ib, rA, rB, t2);
    mfr(c, M_MTW, m) = kw > 0.0f ? 1.0f / kw : 0.0f;
    mfr(c, M_MU, m) = mu;
    mfr(c, M_RT, m) = rsum / float(keep);
    mfr(c, M_REST, m) = e;
    mfr(c, M_LT1, m) = 0.0f; mfr(c, M_LT2, m) = 0.0f; mfr(c, M_LTW, m) = 0.0f;
    if (dbg) {
        float* dm = bd.dbg_man + 8 * size_t(dmo + m);
        dm[0] = __int_as_float(k);
        dm[7] = __int_as_float(keep);
    }
}

// Half size of a part along axis r (add, multiply, abs only, as in the broadphase).
__device__ __forceinline__ float part_half_axis(const Shp& s, int r) {
    return prim_half(s.type, s.d[0], s.d[1], s.d[2], s.R.m[r][0], s.R.m[r][1], s.R.m[r][2]);
}

// The midphase of compound pairs, in the pair frame: the box of part k of body i (body centre at
// `centre`), its centre and its half size along each axis grown by the contact offset; two boxes
// meet when they overlap on every axis, a box reaches the ground when its lowest z is <= 0
// (the broadphase's rule one level down, with the same exact operations on both sides).
__device__ __forceinline__ void part_box(const EnvCtx& c, int i, int k, V3 centre, float delta, V3& pc, V3& ph) {
    const Shp s = part_of(c, i, k, centre);
    pc = s.c;
    ph = v3(part_half_axis(s, 0) + delta, part_half_axis(s, 1) + delta, part_half_axis(s, 2) + delta);
}
__device__ __forceinline__ bool boxes_meet(V3 ca, V3 ha, V3 cb, V3 hb) {
    return (ca.x - ha.x <= cb.x + hb.x) && (cb.x - hb.x <= ca.x + ha.x) && (ca.y - ha.y <= cb.y + hb.y) &&
           (cb.y - hb.y <= ca.y + ha.y) && (ca.z - ha.z <= cb.z + hb.z) && (cb.z - hb.z <= ca.z + ha.z);
}

// S3 + S4 for a chunk of candidates in the compound build (lane per candidate, code < 0: none).
// The candidates expand into items, one per pair of parts (A's parts outer; a
// ground pair pairs the plane with each part of its body) whose grown boxes meet, a primitive
// pair being the one item of its candidate; the items, in this order, are the canonical order
// of the chunk's manifolds.  Phase A: each lane tests its candidate's pairs of parts (a bit
// mask), a scan over the lanes gives each candidate the offset of its first item.  Phase B:
// rounds of G items, item r G + l on lane l, which finds its candidate by a binary search over
// the lanes' offsets and its pair of parts as a set bit of the mask; then each item runs the
// primitive narrowphase and keeps <= 4 points as a manifold of its own under the same capacity
// rule and scans as a chunk of primitive candidates.
__device__ __forceinline__ void compound_chunk(const EnvCtx& c, int code, int k, int& npts, int& nman, bool& overflow,
                                               int li, int g, int G, bool dbg, int dpp, int dpo, int dmo) {
    const Lay& l = c.lay;
    const BatchDev& bd = *c.bd;
    const int n = l.n;
    const float delta = bd.delta;
    // ---- phase A: the item mask of this lane's candidate (bit t: pair of parts t; bit 16: the
    // candidate involves a compound body)
    int mask = 0;
    if (code >= 0) {
        const int a = code & 0xFF, b = code >> 8;
        const bool plane = b == n;
        const int body = plane ? a : b;   // the side whose parts are listed second
        const bool comp = is_compound(c, a) || (!plane && is_compound(c, b));
        if (!comp) {
            mask = 1;
        } else {
            const V3 xa = ldp3(c, a, P_X0);
            const V3 offB = plane ? v3(0.0f, 0.0f, xa.z - bd.plane_z) : ldp3(c, b, P_X0) - xa;
            const int nb = n_parts(c, body);
            const int na = plane ? 1 : n_parts(c, a);
            // one box of each side at a time (the parts' records stay in the caches), so that
            // the test holds few registers
            for (int t = 0; t < na * nb; ++t) {
                const int i = t / nb, j = t - i * nb;
                V3 bc, bh;
                part_box(c, body, j, offB, delta, bc, bh);
                bool meet;
                if (plane) {
                    meet = bc.z - bh.z <= 0.0f;
                } else {
                    V3 ac, ah;
                    part_box(c, a, i, v3(0, 0, 0), delta, ac, ah);
                    meet = boxes_meet(ac, ah, bc, bh);
                }
                if (meet) mask |= 1 << t;
            }
            mask |= 1 << 16;
        }
        if (dbg) {
            int* dp = bd.dbg_pairs + 4 * size_t(dpp + k);
            dp[0] = a; dp[1] = plane ? PLANE : b; dp[2] = 0; dp[3] = comp ? 0x7FFFFFFF : 0;
        }
    }
    int T;
    const int off = group_scan_small<5>(__popc(mask & 0xFFFF), li, g, G, T);
    // ---- phase B: rounds of G items
    const int rounds = wave_max((T + G - 1) / G);
    const int lane0 = g * G;   // first lane of this lane's group
    for (int r = 0; r < rounds; ++r) {
        const int item = r * G + li;
        // owner: the last lane of the group whose first item is <= item (lanes without items
        // share their successor's offset, so the last such lane is the one holding the item)
        int j = 0;
        for (int step = G >> 1; step >= 1; step >>= 1) {
            const int o = __shfl(off, lane0 + j + step);
            if (o <= item) j += step;
        }
        const int ocode = __shfl(code, lane0 + j);
        const int omask = __shfl(mask, lane0 + j);
        const int ooff = __shfl(off, lane0 + j);
        const int ok = __shfl(k, lane0 + j);
        const bool valid = item < T;
        NOut o;
        o.mask = 0;
        o.decision = 0;
        int a = 0, b = 0, t = 0;
        bool plane = false;
        V3 base = v3(0, 0, 0), offB = v3(0, 0, 0);
        if (valid) {
            int m = omask & 0xFFFF;
            for (int q = item - ooff; q > 0; --q) m &= m - 1;
            t = __ffs(m) - 1;
            a = ocode & 0xFF;
            b = ocode >> 8;
            plane = b == n;
            const V3 xa = ldp3(c, a, P_X0);
            if (plane) {
                base = v3(xa.x, xa.y, bd.plane_z);
                offB = v3(0.0f, 0.0f, xa.z - bd.plane_z);
                const Shp sb = part_of(c, a, t, offB);
                atomicAdd(&iptr(c.L + l.SCAL)[16 + STAT_KIND0 + 9 + sb.type], 1);
                np_plane(o, sb, delta);
            } else {
                base = xa;
                offB = ldp3(c, b, P_X0) - xa;
                const int nb = n_parts(c, b);
                const int ia = t / nb;
                const Shp sa = part_of(c, a, ia, v3(0, 0, 0));
                const Shp sb = part_of(c, b, t - ia * nb, offB);
                atomicAdd(&iptr(c.L + l.SCAL)[16 + STAT_KIND0 + 3 * min(sa.type, sb.type) + max(sa.type, sb.type)], 1);
                np_pair(o, sa, sb, delta);
            }
            reduce4(o);
            compact4(o);
        }
        const int on = n_points(o);   // 0 for an invalid item
        int tot;
        const int pre = group_scan_small<3>(on, li, g, G, tot);
        int keep = min(max(l.cap - (npts + pre), 0), on);
        bool ovf = keep < on;
        int mtot;
        const int mpre = group_scan_small<1>(keep > 0 ? 1 : 0, li, g, G, mtot);
        if (keep > 0 && nman + mpre >= l.mcap) { keep = 0; ovf = true; }
        int ktot;
        const int kpre = group_scan_small<3>(keep, li, g, G, ktot);
        overflow |= group_bits(__ballot(ovf), g, G) != 0;
        if (keep > 0) write_rows(c, o, ok, a, b, plane, base, offB, keep, npts + kpre, nman + mpre, t, dbg, dpo, dmo);
        if (valid && dbg) {
            int* dp = bd.dbg_pairs + 4 * size_t(dpp + ok);
            if (keep > 0) atomicAdd(dp + 2, keep);
            if (omask >> 16) {
                if (on > 0) atomicMin(dp + 3, 64 + t);
            } else {
                dp[3] = o.decision;
            }
        }
        npts += ktot;
        int mkept;
        group_scan_small<1>(keep > 0 ? 1 : 0, li, g, G, mkept);
        nman += mkept;
    }
    if (dbg && code >= 0 && (mask >> 16)) {
        // a compound candidate without points: decision 63 (the debug export only)
        __threadfence();
        atomicCAS(bd.dbg_pairs + 4 * size_t(dpp + k) + 3, 0x7FFFFFFF, 63);
    }
}

}  // namespace

// ============================================================================= step kernel
// The step of every tile of the work list; `lds` is the workgroup's dynamic LDS.
// ONE: every tile of the launch holds a single env served by all 64 lanes, so the env's sizes
// and offsets are wavefront-uniform (scalar registers) and the group arithmetic folds away.
// Net contact impulse on each dynamic body, summed into the bounding-box plane (free after the
// broadphase; 3 of its 6 n words): a lane per body walks its block list (colour order, built for
// the warm start) and adds, for each manifold it belongs to, the normal impulses of its points,
// then the patch's two tangent impulses (added on side B, subtracted on side A; the twist is a
// torque and is left out; static bodies keep zero).  Run once after the sweeps of every substep
// but the last, and once after the velocity and restitution passes: the sum over substeps of
// each substep's final multipliers.
// Whether the batch accumulates contact forces, read afresh at each use (a volatile load) so the
// flag never holds a register across the step's phases.
__device__ __forceinline__ bool forces_on(const EnvCtx& c) {
    return *reinterpret_cast<float* const volatile*>(&c.bd->forces) != nullptr;
}
__device__ __forceinline__ void accumulate_forces(const EnvCtx& c, int nn, int li, int G) {
    const Lay& l = c.lay;
    const int n = l.n;
    float* F = c.L + l.AABB;
    const int* OFF = iptr(c.L + l.CAND);
    const uint16_t* ENT = reinterpret_cast<const uint16_t*>(OFF + l.n + 1);
    for (int i = li; i < nn; i += G) {
        if (!is_dyn(c, i)) continue;
        V3 f = v3(F[i], F[n + i], F[2 * n + i]);
        for (int e = OFF[i]; e < OFF[i + 1]; ++e) {
            const int ent = ENT[e];
            const int blk = ent & 0x7FFF;
            if (blk < l.nj) continue;
            const bool sideB = (ent >> 15) != 0;
            const int m = blk - l.nj;
            int a, b, first, cnt;
            man_header(c, m, a, b, first, cnt);
            for (int k = first; k < first + cnt; ++k) {
                const V3 Pn = pr(c, R_LN, k) * pr3(c, R_N, k);
                f = sideB ? f + Pn : f - Pn;
            }
            const V3 t1 = mf3(c, M_T1, m);
            const V3 Pt = mf(c, M_LT1, m) * t1 + mf(c, M_LT2, m) * cross3(mf3(c, M_NB, m), t1);
            f = sideB ? f + Pt : f - Pt;
        }
        F[i] = f.x; F[n + i] = f.y; F[2 * n + i] = f.z;
    }
}

// ----------------------------------------------------------------------------- S4b contact cache
// Key of manifold m, increasing in canonical order: (lower body, partner, pair of parts), the
// ground plane after every partner of its body.
__device__ __forceinline__ int man_key(const EnvCtx& c, int m) {
    const int ab = iptr(c.L + c.lay.MAN + m * M_WORDS)[M_AB];
    const int a = ab & 0xFF, b = (ab >> 8) & 0xFF, part = (ab >> 16) & 0xF;
    return ((a != 0xFF ? (a << 8) | b : (b << 8) | 0xFF) << 4) | part;
}
// Initial impulses from the last step's cache (lane per manifold): a manifold whose pair is
// cached takes, for each point, the normal impulse of the nearest cached point of that pair
// (positions in body B's frame at the step start, squared distance below warm_radius^2, the
// first cached point on ties), and the cached tangential impulse vector projected on its new
// tangents, and the cached twist impulse.  The cached keys are staged in the candidate area
// (free between the row setup and the block lists) for a binary search per lane.
__device__ __forceinline__ void warm_from_cache(const EnvCtx& c, int nman, int li, int G) {
    const BatchDev& bd = *c.bd;
    __threadfence();   // this env's cache may have been written by this wave's previous step
    const int nc = gldi(bd.cache_hdr + 2 * c.env);
    const int* CM = reinterpret_cast<const int*>(bd.cache_man) + size_t(bd.cache_man_off[c.env]) * CM_WORDS;
    const float* CP = bd.cache_pt + size_t(bd.cache_pt_off[c.env]) * CP_WORDS;
    int* KEYS = iptr(c.L + c.lay.CAND);
    for (int k = li; k < nc; k += G) KEYS[k] = gldi(CM + k * CM_WORDS);
    wave_sync();
    const float r2 = bd.warm_radius * bd.warm_radius;
    for (int m = li; m < nman; m += G) {
        const int key = man_key(c, m);
        int lo = 0, hi = nc;
        while (lo < hi) {
            const int mid = (lo + hi) / 2;
            if (KEYS[mid] < key) lo = mid + 1; else hi = mid;
        }
        if (lo == nc || KEYS[lo] != key) continue;
        const int* rec = CM + lo * CM_WORDS;
        int rw[6];
        for (int w = 1; w < 6; ++w) rw[w] = gldi(rec + w);
        const int cfc = rw[1];
        const int cfirst = cfc & 0xFFFF, ccount = cfc >> 16;
        const V3 pt = v3(__int_as_float(rw[2]), __int_as_float(rw[3]), __int_as_float(rw[4]));
        int a, b, first, cnt;
        man_header(c, m, a, b, first, cnt);
        const M3 RB = rotm(ldp4(c, b, P_Q0));
        for (int k = first; k < first + cnt; ++k) {
            const V3 rl = mulTv(RB, pr3(c, R_RB, k));
            float best = r2;
            int bj = -1;
            for (int j = 0; j < ccount; ++j) {
                const float* q = CP + (cfirst + j) * CP_WORDS;
                const V3 d = rl - v3(gld(q), gld(q + 1), gld(q + 2));
                const float d2 = dot3(d, d);
                if (d2 < best) { best = d2; bj = j; }
            }
            if (bj >= 0) pr(c, R_LN, k) = gld(CP + (cfirst + bj) * CP_WORDS + 3);
        }
        const V3 t1 = mf3(c, M_T1, m);
        mfr(c, M_LT1, m) = dot3(pt, t1);
        mfr(c, M_LT2, m) = dot3(pt, cross3(mf3(c, M_NB, m), t1));
        mfr(c, M_LTW, m) = __int_as_float(rw[5]);
    }
    wave_sync();
}
// The cache for the next step (lane per manifold): every manifold of this step with its final
// impulses and its points' positions in body B's frame; a step that went non-finite leaves an
// empty cache.
__device__ __forceinline__ void write_cache(const EnvCtx& c, int nman, int npts, bool bad, int li, int G) {
    const BatchDev& bd = *c.bd;
    int* CM = reinterpret_cast<int*>(bd.cache_man) + size_t(bd.cache_man_off[c.env]) * CM_WORDS;
    float* CP = bd.cache_pt + size_t(bd.cache_pt_off[c.env]) * CP_WORDS;
    if (li == 0) {
        gsti(bd.cache_hdr + 2 * c.env, bad ? 0 : nman);
        gsti(bd.cache_hdr + 2 * c.env + 1, bad ? 0 : npts);
    }
    if (bad) return;
    for (int m = li; m < nman; m += G) {
        int a, b, first, cnt;
        man_header(c, m, a, b, first, cnt);
        const V3 t1 = mf3(c, M_T1, m);
        const V3 pt = mf(c, M_LT1, m) * t1 + mf(c, M_LT2, m) * cross3(mf3(c, M_NB, m), t1);
        int* rec = CM + m * CM_WORDS;
        gsti(rec, man_key(c, m));
        gsti(rec + 1, first | (cnt << 16));
        gsti(rec + 2, __float_as_int(pt.x)); gsti(rec + 3, __float_as_int(pt.y)); gsti(rec + 4, __float_as_int(pt.z));
        gsti(rec + 5, __float_as_int(mf(c, M_LTW, m)));
        const M3 RB = rotm(ldp4(c, b, P_Q0));
        for (int k = first; k < first + cnt; ++k) {
            const V3 rl = mulTv(RB, pr3(c, R_RB, k));
            float* q = CP + k * CP_WORDS;
            const float ln = pr(c, R_LN, k);
            gst(q, rl.x); gst(q + 1, rl.y); gst(q + 2, rl.z); gst(q + 3, ln);
        }
    }
}
__device__ __forceinline__ bool warm_on(const EnvCtx& c) {
    return *reinterpret_cast<int* const volatile*>(&c.bd->cache_hdr) != nullptr;
}

// Per-phase clock (a build flag, MS_PHASE_CLOCK, off in the library's default build): each
// wavefront reads the shader clock at the phase boundaries of the step and adds the cycles spent
// in each phase to bd.phase_clock[phase] at the end of its launch (wave-cycles, stalls included).
enum { PH_LOAD, PH_POSE, PH_BROAD, PH_NARROW, PH_CACHE, PH_COLOUR, PH_LISTS, PH_SUBSTART, PH_BIAS, PH_WARMJ,
       PH_SWEEP, PH_FORCES, PH_INTEG, PH_VEL, PH_GUARD, PH_STORE, N_PHASES };
#ifdef MS_PHASE_CLOCK
#define PHASE(k)                                              \
    do {                                                      \
        const uint64_t t_ = __builtin_amdgcn_s_memtime();     \
        ph_acc[k] += t_ - ph_t;                               \
        ph_t = t_;                                            \
        refresh_lay();                                        \
    } while (0)
#else
#define PHASE(k)        \
    do {                \
        refresh_lay();  \
    } while (0)
#endif

// FEAT: the optional parts the build carries.  FEAT_OPT: the optional phases (contact-force
// readout, contact cache); FEAT_COMP: compound bodies as well (their part-pair narrowphase and
// boxes).  The default builds leave both out entirely, so that they cost the plain step no
// registers, and the compound build is apart from the optional-phase one for the same reason.
enum { FEAT_OPT = 1, FEAT_COMP = 2 };
template <bool ONE, int FEAT>
__device__ __forceinline__ void step_tile(float* lds, const BatchDev* __restrict__ batches, const Tile tile,
                                          const TileEnv* __restrict__ tenv, int n_steps, int lane) {
    constexpr bool OPT = (FEAT & FEAT_OPT) != 0;
    constexpr bool COMP = (FEAT & FEAT_COMP) != 0;
    {
#ifdef MS_PHASE_CLOCK
        uint64_t ph_acc[N_PHASES] = {};
        uint64_t ph_t = __builtin_amdgcn_s_memtime();
#endif
        const int G = ONE ? WAVE : tile.lanes;
        const int g = ONE ? 0 : lane / G, li = ONE ? lane : lane % G;
        EnvCtx c;
        c.active = ONE ? true : g < tile.count;
        TileEnv te = ONE ? tenv[tile.first] : (c.active ? tenv[tile.first + g] : tenv[tile.first]);
        c.bd = &batches[te.batch];
        c.env = te.env;
        c.L = lds + te.lds_off;
        c.lay = make_lay(te.n, te.nj, te.cap, te.mcap);
        // In the general build the layout is per group (vector registers): it is re-derived
        // from the env's four sizes at every phase boundary, opaque to the optimiser, so that
        // its twenty-odd offsets are live within a phase instead of across the launch.
        const int lay_n = te.n, lay_nj = te.nj, lay_cap = te.cap, lay_mcap = te.mcap;
        auto refresh_lay = [&]() {
            if constexpr (!ONE)
                c.lay = make_lay(opaque_lane(lay_n), opaque_lane(lay_nj), opaque_lane(lay_cap), opaque_lane(lay_mcap));
        };
        const BatchDev& bd = *c.bd;
        const Lay& l = c.lay;
        const int n = l.n;
        const int nj = l.nj;
        const int nA = c.active ? n : 0;    // bodies this lane's group owns
        const int njA = c.active ? nj : 0;
        c.b0 = bd.body_off[c.env];
        c.j0 = bd.joint_off[c.env];
        int* SC = iptr(c.L + l.SCAL);
        const int B = bd.B;

        // ------------------------------------------------------------- load (once per launch)
        // every HBM value of a body first (16 loads in flight at once), then its LDS records
        for (int i = li; i < nA; i += G) {
            const int gi = c.b0 + i;
            float st[13];
            for (int r = 0; r < 3; ++r) st[r] = gld(bd.pos + r * B + gi);
            for (int r = 0; r < 4; ++r) st[3 + r] = gld(bd.quat + r * B + gi);
            for (int r = 0; r < 3; ++r) st[7 + r] = gld(bd.vel + r * B + gi);
            for (int r = 0; r < 3; ++r) st[10 + r] = gld(bd.angvel + r * B + gi);
            const float4 p0 = gld4(bd.bpar + gi), p1 = gld4(bd.bpar + B + gi), p2 = gld4(bd.bpar + 2 * B + gi);
            for (int r = 0; r < 3; ++r) pose_rec(c, i)[P_X0 + r] = st[r];
            for (int r = 0; r < 4; ++r) pose_rec(c, i)[P_QC + r] = st[3 + r];
            for (int r = 0; r < 3; ++r) body_rec(c, i)[B_V + r] = st[7 + r];
            for (int r = 0; r < 3; ++r) body_rec(c, i)[B_W + r] = st[10 + r];
            int sh = __float_as_int(p0.x);
            iptr(c.L + l.SH)[i] = sh;
            bool dyn = !((sh >> 8) & 1);
            body_rec(c, i)[B_IM] = dyn ? p0.y : 0.0f;
            c.L[l.MU + i] = p0.z;
            c.L[l.EE + i] = p0.w;
            c.L[l.DIM + i] = p1.x; c.L[l.DIM + n + i] = p1.y; c.L[l.DIM + 2 * n + i] = p1.z;
            c.L[l.IB + i] = dyn ? p2.x : 0.0f;
            c.L[l.IB + n + i] = dyn ? p2.y : 0.0f;
            c.L[l.IB + 2 * n + i] = dyn ? p2.z : 0.0f;
            stp3(c, i, P_DX, v3(0, 0, 0));
        }
        for (int j = li; j < njA; j += G) {
            const float* src = bd.jrec + size_t(c.j0 + j) * JREC;
            float jr[21];
            for (int w = 0; w < 21; ++w) jr[w] = gld(src + w);
            const float tg = gld(bd.targets + c.j0 + j);
            float* J = jrec(c, j);
            for (int w = 0; w < 18; ++w) J[w] = jr[w];
            J[J_TG] = tg;
            J[J_TYP] = jr[18];
            J[J_LO] = jr[19];
            J[J_HI] = jr[20];
        }
        if (c.active && li == 0) SC[SC_STATUS] = gldi(bd.status + c.env);
        for (int k = li; k < (c.active ? NSTAT : 0); k += G) SC[16 + k] = 0;
        wave_sync();
        // jointed-partner masks (parent-child pairs never collide)
        for (int i = li; i < nA; i += G) {
            uint64_t m = 0;
            for (int j = 0; j < nj; ++j) {
                const int* J = reinterpret_cast<const int*>(jrec(c, j));
                int pa = J[J_PA], ch = J[J_CH];
                if (pa < 0) continue;
                if (pa == i) m |= uint64_t(1) << ch;
                if (ch == i) m |= uint64_t(1) << pa;
            }
            iptr(c.L + l.JM)[2 * i] = int(uint32_t(m));
            iptr(c.L + l.JM)[2 * i + 1] = int(uint32_t(m >> 32));
        }
        wave_sync();
        PHASE(PH_LOAD);

        const int li_outer = li;
        for (int step = 0; step < n_steps; ++step) {
            // the lane index, opaque to the optimiser at each step: lane-dependent addresses are
            // formed where they are used instead of once per launch and held (spilled) across it
            const int li = opaque_lane(li_outer);
            const bool frozen = !c.active || (SC[SC_STATUS] & 1);
            const int nn = frozen ? 0 : n;
            const int S = bd.S, K = bd.K;
            const float h = bd.dt / float(S);
            const bool dbg = bd.dbg_pairs != nullptr && step == n_steps - 1 && !frozen;
            if (bd.dbg_pairs != nullptr && step == n_steps - 1 && frozen && c.active && li == 0) {
                int* dc = bd.dbg_counts + 4 * c.env;
                dc[0] = 0; dc[1] = 0; dc[2] = 0; dc[3] = 0;
            }
            wave_sync();

            // --------------------------------------------------------- S0 + S1
            for (int i = li; i < nn; i += G) {
                V3 x0 = ldp3(c, i, P_X0) + ldp3(c, i, P_DX);
                stp3(c, i, P_X0, x0);
                stp4(c, i, P_Q0, ldp4(c, i, P_QC));
                stp3(c, i, P_DX, v3(0, 0, 0));
                stp4(c, i, P_DQ, Qt{1.0f, 0.0f, 0.0f, 0.0f});
                st3(c.L, l.V0, n, i, ldv(c, i));
                st3(c.L, l.W0, n, i, ldw(c, i));
                // world inverse inertia R diag(I^-1) R^T from the step-start orientation
                M3 R = rotm(ldp4(c, i, P_Q0));
                float d0 = c.L[l.IB + i], d1 = c.L[l.IB + n + i], d2 = c.L[l.IB + 2 * n + i];
                float Iw[3][3];
                for (int p = 0; p < 3; ++p)
                    for (int q = p; q < 3; ++q)
                        Iw[p][q] = R.m[p][0] * d0 * R.m[q][0] + R.m[p][1] * d1 * R.m[q][1] + R.m[p][2] * d2 * R.m[q][2];
                float* Iwr = body_rec(c, i) + B_IW;
                Iwr[0] = Iw[0][0]; Iwr[1] = Iw[1][1]; Iwr[2] = Iw[2][2];
                Iwr[3] = Iw[0][1]; Iwr[4] = Iw[0][2]; Iwr[5] = Iw[1][2];
                body_aabb<COMP>(c, i);
                iptr(c.L + l.CM)[2 * i] = 0;
                iptr(c.L + l.CM)[2 * i + 1] = 0;
            }
            // joint impulses start every step from zero (no cross-step warm start)
            for (int j = li; j < (frozen ? 0 : nj); j += G) {
                float* J = jrec(c, j);
                for (int w = J_LP; w < J_LL + 2; ++w) J[w] = 0.0f;
            }
            wave_sync();

            PHASE(PH_POSE);
            // --------------------------------------------------------- S2 candidate pairs
            const int P = frozen ? 0 : l.P;
            int ncand = 0;
            if (G == WAVE) {
                // one env per wave: lane a tests a against every later body b (b's box read by
                // all lanes at once) into a bit mask, then writes its pairs b ascending and the
                // plane last at its offset in a scan over lanes: canonical order
                uint16_t* CAND = reinterpret_cast<uint16_t*>(c.L + l.CAND);
                const int nw = __builtin_amdgcn_readfirstlane(nn);
                const int a = li;
                const bool act = a < nw;
                const float* AB = c.L + l.AABB;
                V3 amin = v3(0, 0, 0), amax = v3(0, 0, 0);
                uint64_t jm = 0;
                bool dyn_a = false;
                if (act) {
                    amin = v3(AB[a], AB[n + a], AB[2 * n + a]);
                    amax = v3(AB[3 * n + a], AB[4 * n + a], AB[5 * n + a]);
                    const int* JMi = iptr(c.L + l.JM);
                    jm = uint64_t(uint32_t(JMi[2 * a])) | (uint64_t(uint32_t(JMi[2 * a + 1])) << 32);
                    dyn_a = is_dyn(c, a);
                }
                const uint64_t dynm = __ballot(dyn_a);
                uint64_t mask = 0;
                for (int b = 1; b < nw; ++b) {
                    const V3 bmin = v3(AB[b], AB[n + b], AB[2 * n + b]);
                    const V3 bmax = v3(AB[3 * n + b], AB[4 * n + b], AB[5 * n + b]);
                    const bool ov = b > a && (dyn_a || ((dynm >> b) & 1)) && !((jm >> b) & 1) &&
                                    (amin.x <= bmax.x && bmin.x <= amax.x) && (amin.y <= bmax.y && bmin.y <= amax.y) &&
                                    (amin.z <= bmax.z && bmin.z <= amax.z);
                    if (ov) mask |= uint64_t(1) << b;
                }
                const bool pl = act && bd.plane && dyn_a && amin.z <= bd.plane_z;
                const int cnt = __popcll(mask) + (pl ? 1 : 0);
                int tot;
                int o = group_scan_small<7>(cnt, li, 0, WAVE, tot);
                while (mask) {
                    const int b = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    CAND[o++] = uint16_t(a | (b << 8));
                }
                if (pl) CAND[o] = uint16_t(a | (n << 8));
                ncand = tot;
            } else {
                const int nch = wave_max((P + G - 1) / G);
                uint16_t* CAND = reinterpret_cast<uint16_t*>(c.L + l.CAND);
                const int* JMi = iptr(c.L + l.JM);
                for (int ch = 0; ch < nch; ++ch) {
                    int k = ch * G + li;
                    bool cand = false;
                    int a = 0, b = 0;
                    if (k < P) {
                        pair_of(k, n, a, b);
                        if (b == n) {
                            cand = bd.plane && is_dyn(c, a) && c.L[l.AABB + 2 * n + a] <= bd.plane_z;
                        } else {
                            bool jointed = b < 32 ? ((JMi[2 * a] >> b) & 1) : ((JMi[2 * a + 1] >> (b - 32)) & 1);
                            cand = (is_dyn(c, a) || is_dyn(c, b)) && !jointed && aabb_overlap(c, a, b);
                        }
                    }
                    uint64_t gb = group_bits(__ballot(cand), g, G);
                    if (cand) CAND[ncand + prefix_in_group(gb, li)] = uint16_t(a | (b << 8));
                    ncand += __popcll(gb);
                }
            }
            wave_sync();

            PHASE(PH_BROAD);
            // --------------------------------------------------------- S3 + S4 narrowphase, rows
            int npts = 0, nman = 0;
            bool overflow = false;
            {
                const int nch = wave_max((ncand + G - 1) / G);
                const uint16_t* CAND = reinterpret_cast<const uint16_t*>(c.L + l.CAND);
                const float delta = bd.delta;
                int dpo = 0, dmo = 0, dpp = 0;
                if (dbg) { dpp = bd.dbg_pair_off[c.env]; dpo = bd.dbg_pt_off[c.env]; dmo = bd.dbg_man_off[c.env]; }
                for (int ch = 0; ch < nch; ++ch) {
                    int k = ch * G + li;
                    if constexpr (COMP) {
                        // the compound build has the one narrowphase path of part-pair items
                        // (a chunk without compounds is one item per candidate)
                        const int code = k < ncand ? int(CAND[k]) : -1;
                        compound_chunk(c, code, k, npts, nman, overflow, li, g, G, dbg, dpp, dpo, dmo);
                        continue;
                    }
                    NOut o;
                    int a = 0, b = 0;
                    bool plane = false;
                    V3 base, offB;
                    np_candidate(c, k < ncand ? int(CAND[k]) : -1, o, a, b, plane, base, offB);
                    int tot;
                    const int on = n_points(o);   // 0..4
                    int pre = group_scan_small<3>(on, li, g, G, tot);
                    int keep = min(max(l.cap - (npts + pre), 0), on);
                    bool ovf = keep < on;
                    int mtot;
                    int mpre = group_scan_small<1>(keep > 0 ? 1 : 0, li, g, G, mtot);
                    if (keep > 0 && nman + mpre >= l.mcap) { keep = 0; ovf = true; }
                    int ktot;
                    int kpre = group_scan_small<3>(keep, li, g, G, ktot);
                    int m_idx = nman + mpre;
                    int first = npts + kpre;
                    overflow |= group_bits(__ballot(ovf), g, G) != 0;
                    if (k < ncand && dbg) {
                        int* dp = bd.dbg_pairs + 4 * size_t(dpp + k);
                        dp[0] = a; dp[1] = plane ? PLANE : b; dp[2] = keep; dp[3] = o.decision;
                    }
                    if (keep > 0) write_rows(c, o, k, a, b, plane, base, offB, keep, first, m_idx, 0, dbg, dpo, dmo);
                    npts += ktot;
                    int mkept;
                    group_scan_small<1>(keep > 0 ? 1 : 0, li, g, G, mkept);
                    nman += mkept;
                }
            }
            if (!frozen && li == 0) {
                SC[SC_NCAND] = ncand;
                SC[SC_NPTS] = npts;
                SC[SC_NMAN] = nman;
                if (overflow) SC[SC_STATUS] |= 2;
                SC[16 + STAT_STEPS] += 1;
                SC[16 + STAT_POINTS] += npts;
                SC[16 + STAT_MANIFOLDS] += nman;
            }
            wave_sync();
            PHASE(PH_NARROW);
            // --------------------------------------------------------- S4b cross-step warm start
            // (the batch's flag is re-read at each use, a volatile scalar load, so that it holds
            // no register through the substeps)
            if (OPT && !frozen && warm_on(c)) warm_from_cache(c, nman, li, G);

            PHASE(PH_CACHE);
            // --------------------------------------------------------- S5 colouring
            if (G == WAVE) {
                if (!frozen) colour_env_wave(c);
            } else if (!frozen && li == 0) {
                colour_env(c, G);
            }
            wave_sync();
            if (!frozen && li == 0) SC[16 + STAT_COLOURS] += SC[SC_NCOL];
            wave_sync();
            const int ns = frozen ? 0 : SC[SC_NSCHED];
            const int njs = frozen ? 0 : SC[SC_NJSCHED];
            const int ns_max = wave_max(ns), njs_max = wave_max(njs);
            const int JI = bd.JI;
            const bool pipe = __ballot(c.active && nj > 0) == 0;   // no joints anywhere in the wave
            const int nmanA = frozen ? 0 : SC[SC_NMAN];

            PHASE(PH_COLOUR);
            // --------------------------------------------------------- S6 substeps
            if (OPT && forces_on(c)) {
                for (int i = li; i < nn; i += G) {
                    c.L[l.AABB + i] = 0.0f; c.L[l.AABB + n + i] = 0.0f; c.L[l.AABB + 2 * n + i] = 0.0f;
                }
            }
            const float ldmp = 1.0f / (1.0f + h * bd.lin_damp);
            const float admp = 1.0f / (1.0f + h * bd.ang_damp);
            // warm start body by body: fused with gravity in joint-free waves, after the joint pass
            // in the others
            if (S > 1 || (OPT && (warm_on(c) || forces_on(c)))) {   // warm start, force sums
                if (G == WAVE) build_body_lists_wave(c, nn, nmanA, li);
                else build_body_lists(c, nn, nmanA, li, G);
                wave_sync();
            }
            PHASE(PH_LISTS);
            for (int s = 0; s < S; ++s) {
                // warm start: the previous substep's impulses, or the cached ones in the first
                const bool gather = pipe && (s > 0 || (OPT && !frozen && warm_on(c)));
                for (int i = li; i < nn; i += G)
                    if (is_dyn(c, i)) body_substep_start(c, i, h, ldmp, admp, gather);
                PHASE(PH_SUBSTART);
                bias_pass(c, nmanA, h, false, li, G);
                for (int j = li; j < (frozen ? 0 : nj); j += G) joint_prep(c, j, h);
                wave_sync();
                PHASE(PH_BIAS);
                if ((s > 0 || (OPT && !frozen && warm_on(c))) && !pipe) {   // waves with joints: gathered per body once the joint pass has run
                    for (int i = li; i < nn; i += G)
                        if (is_dyn(c, i)) body_warm_gather(c, i);
                    wave_sync();
                }
                PHASE(PH_WARMJ);
                for (int it = 0; it < K; ++it) {
                    for (int jx = 1; jx < JI; ++jx) run_schedule<OP_JOINT, false>(c, l.JSCHED, njs, njs_max, h, li);
                    (pipe && G >= 2 ? run_schedule_pairs(c, l.SCHED, ns, ns_max, li, G) : pipe ? run_schedule<OP_SOLVE, true>(c, l.SCHED, ns, ns_max, h, li) : run_schedule<OP_SOLVE, false>(c, l.SCHED, ns, ns_max, h, li));
                }
                PHASE(PH_SWEEP);
                if (OPT && s + 1 < S && forces_on(c)) {
                    wave_sync();
                    accumulate_forces(c, nn, li, G);
                }
                PHASE(PH_FORCES);
                // integrate the offsets from the step-start pose
                for (int i = li; i < nn; i += G) {
                    if (!is_dyn(c, i)) continue;
                    V3 v = ldv(c, i), w = ldw(c, i);
                    stp3(c, i, P_DX, ldp3(c, i, P_DX) + h * v);
                    Qt d = ldp4(c, i, P_DQ);
                    Qt e = qmul(Qt{0.0f, w.x, w.y, w.z}, d);
                    float hh = 0.5f * h;
                    d = qnorm(Qt{d.w + hh * e.w, d.x + hh * e.x, d.y + hh * e.y, d.z + hh * e.z});
                    stp4(c, i, P_DQ, d);
                    stp4(c, i, P_QC, qnorm(qmul(d, ldp4(c, i, P_Q0))));
                }
                wave_sync();
                PHASE(PH_INTEG);
            }
            // --------------------------------------------------------- S7
            if (bd.V > 0) {
                bias_pass(c, nmanA, h, true, li, G);
                for (int j = li; j < (frozen ? 0 : nj); j += G) joint_prep(c, j, h);
                wave_sync();
            }
            for (int it = 0; it < bd.V; ++it) (pipe && G >= 2 ? run_schedule_pairs(c, l.SCHED, ns, ns_max, li, G) : pipe ? run_schedule<OP_VSOLVE, true>(c, l.SCHED, ns, ns_max, h, li) : run_schedule<OP_VSOLVE, false>(c, l.SCHED, ns, ns_max, h, li));
            run_schedule<OP_REST, false>(c, l.SCHED, ns, ns_max, h, li);
            PHASE(PH_VEL);

            // --------------------------------------------------------- S8 non-finite guard
            bool bad = false;
            for (int i = li; i < nn; i += G) {
                V3 x = ldp3(c, i, P_X0) + ldp3(c, i, P_DX);
                Qt q = ldp4(c, i, P_QC);
                V3 v = ldv(c, i), w = ldw(c, i);
                float vals[13] = {x.x, x.y, x.z, q.w, q.x, q.y, q.z, v.x, v.y, v.z, w.x, w.y, w.z};
                for (int r = 0; r < 13; ++r) bad |= !isfinite(vals[r]);
            }
            bool anybad = group_bits(__ballot(bad), g, G) != 0;
            if (anybad) {
                for (int i = li; i < nn; i += G) {
                    stp3(c, i, P_DX, v3(0, 0, 0));
                    stp4(c, i, P_QC, ldp4(c, i, P_Q0));
                    stv(c, i, ld3(c.L, l.V0, n, i));
                    stw(c, i, ld3(c.L, l.W0, n, i));
                }
                if (li == 0) SC[SC_STATUS] |= 1;
            }
            wave_sync();
            if (OPT && !frozen && warm_on(c)) write_cache(c, nmanA, SC[SC_NPTS], anybad, li, G);
            // --------------------------------------------------------- contact forces
            // the step's contact impulses / dt, written for the last step of the launch (zero for
            // a frozen env or a step that went non-finite)
            if (OPT && step == n_steps - 1 && forces_on(c)) {
                if (!anybad) accumulate_forces(c, nn, li, G);
                const float idt = 1.0f / bd.dt;
                for (int i = li; i < nA; i += G) {
                    V3 f = v3(0, 0, 0);
                    if (!frozen && !anybad) f = idt * v3(c.L[l.AABB + i], c.L[l.AABB + n + i], c.L[l.AABB + 2 * n + i]);
                    const int gi = c.b0 + i;
                    gst(bd.forces + gi, f.x); gst(bd.forces + B + gi, f.y); gst(bd.forces + 2 * B + gi, f.z);
                }
            }
            wave_sync();
            // --------------------------------------------------------- debug export
            if (dbg) {
                int dpo = bd.dbg_pt_off[c.env], dmo = bd.dbg_man_off[c.env];
                for (int k = li; k < npts; k += G) bd.dbg_pts[8 * size_t(dpo + k) + 7] = pr(c, R_LN, k);
                const uint16_t* BC = reinterpret_cast<const uint16_t*>(c.L + l.BCOL);
                for (int m = li; m < nman; m += G) {
                    float* dm = bd.dbg_man + 8 * size_t(dmo + m);
                    dm[1] = __int_as_float(int(BC[nj + m]));
                    dm[2] = mf(c, M_LT1, m); dm[3] = mf(c, M_LT2, m); dm[4] = mf(c, M_LTW, m);
                    dm[5] = mf(c, M_MU, m); dm[6] = mf(c, M_RT, m);
                }
                if (li == 0) {
                    int* dc = bd.dbg_counts + 4 * c.env;
                    dc[0] = ncand; dc[1] = npts; dc[2] = nman; dc[3] = SC[SC_NCOL];
                }
            }
            PHASE(PH_GUARD);
        }
        wave_sync();
        // ------------------------------------------------------------- store
        // a body's LDS words first, then its HBM stores; counters by 64-bit atomic adds (no read
        // of the old value)
        for (int i = li; i < nA; i += G) {
            const int gi = c.b0 + i;
            const V3 x = ldp3(c, i, P_X0) + ldp3(c, i, P_DX);
            const Qt q = ldp4(c, i, P_QC);
            const V3 v = ldv(c, i), w = ldw(c, i);
            gst(bd.pos + gi, x.x); gst(bd.pos + B + gi, x.y); gst(bd.pos + 2 * B + gi, x.z);
            gst(bd.quat + gi, q.w); gst(bd.quat + B + gi, q.x); gst(bd.quat + 2 * B + gi, q.y); gst(bd.quat + 3 * B + gi, q.z);
            gst(bd.vel + gi, v.x); gst(bd.vel + B + gi, v.y); gst(bd.vel + 2 * B + gi, v.z);
            gst(bd.angvel + gi, w.x); gst(bd.angvel + B + gi, w.y); gst(bd.angvel + 2 * B + gi, w.z);
        }
        if (c.active && li == 0) gsti(bd.status + c.env, SC[SC_STATUS]);
        for (int k = li; k < (c.active ? NSTAT : 0); k += G) gadd64(bd.stats + NSTAT * c.env + k, (long long)SC[16 + k]);
        wave_sync();
        PHASE(PH_STORE);
#ifdef MS_PHASE_CLOCK
        if (lane == 0 && bd.phase_clock)
            for (int k = 0; k < N_PHASES; ++k) atomicAdd(&bd.phase_clock[k], (unsigned long long)ph_acc[k]);
#endif
    }
}

// Workgroups of one wavefront walking the tile list.
template <bool ONE, int FEAT>
__device__ __forceinline__ void step_tiles(float* lds, const BatchDev* __restrict__ batches,
                                           const Tile* __restrict__ tiles, int n_tiles,
                                           const TileEnv* __restrict__ tenv, int n_steps) {
    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x)
        step_tile<ONE, FEAT>(lds, batches, tiles[t], tenv, n_steps, opaque_lane(int(threadIdx.x)));
}

// One launch for every tile of a batch: workgroups of BIN_WAVES wavefronts, one bin each; wave w
// runs tile w of its bin in the bin's LDS at that tile's offset (the scalar-env build for a tile
// of one env on all 64 lanes, the general build otherwise).  Waves of a bin share nothing
// but the allocation (every env lives in one wave), so they need no barrier.
template <int FEAT>
__device__ __forceinline__ void step_bins(const BatchDev* __restrict__ batches, const Tile* __restrict__ tiles,
                                          const Bin* __restrict__ bins, int n_bins, const TileEnv* __restrict__ tenv,
                                          int n_steps) {
    extern __shared__ float lds[];
    const int wave = int(threadIdx.x) / WAVE;
    const int b = int(blockIdx.x);
    if (b >= n_bins) return;
    const Bin& bin = bins[b];
    if (wave >= bin.count) return;
    const Tile tile = tiles[bin.tile[wave]];
    const int lane = int(threadIdx.x) & (WAVE - 1);
    if (tile.lanes == WAVE && tile.count == 1) step_tile<true, FEAT>(lds + bin.off[wave], batches, tile, tenv, n_steps, lane);
    else step_tile<false, FEAT>(lds + bin.off[wave], batches, tile, tenv, n_steps, lane);
}

// Builds of the same step: any tiling with unconstrained register allocation (small envs, where
// the wave count is bounded by LDS anyway) or capped at 256 registers per lane (two waves per
// SIMD); the same two for launches whose tiles all hold one env served by the whole wavefront;
// and the bins launch.  The planner / tuner picks one per LDS class.  The *_opt twins carry the
// optional phases (batches with contact forces or the contact cache on), the *_comp ones those
// and compound bodies.
#define MS_TILE_KERNEL(NAME, ONE, FEAT, ATTR)                                                                   \
    extern "C" __global__ void __launch_bounds__(64) ATTR NAME(const BatchDev* __restrict__ batches,            \
                                                               const Tile* __restrict__ tiles, int n_tiles,    \
                                                               const TileEnv* __restrict__ tenv, int n_steps) { \
        extern __shared__ float lds[];                                                                         \
        step_tiles<ONE, FEAT>(lds, batches, tiles, n_tiles, tenv, n_steps);                                     \
    }
#define MS_W2 __attribute__((amdgpu_waves_per_eu(2)))
MS_TILE_KERNEL(ms_step_kernel, false, 0, )
MS_TILE_KERNEL(ms_step_kernel_w2, false, 0, MS_W2)
MS_TILE_KERNEL(ms_step_kernel_one, true, 0, )
MS_TILE_KERNEL(ms_step_kernel_one_w2, true, 0, MS_W2)
MS_TILE_KERNEL(ms_step_kernel_opt, false, FEAT_OPT, )
MS_TILE_KERNEL(ms_step_kernel_w2_opt, false, FEAT_OPT, MS_W2)
MS_TILE_KERNEL(ms_step_kernel_one_opt, true, FEAT_OPT, )
MS_TILE_KERNEL(ms_step_kernel_one_w2_opt, true, FEAT_OPT, MS_W2)
MS_TILE_KERNEL(ms_step_kernel_comp, false, FEAT_OPT | FEAT_COMP, )
MS_TILE_KERNEL(ms_step_kernel_w2_comp, false, FEAT_OPT | FEAT_COMP, MS_W2)
MS_TILE_KERNEL(ms_step_kernel_one_comp, true, FEAT_OPT | FEAT_COMP, )
MS_TILE_KERNEL(ms_step_kernel_one_w2_comp, true, FEAT_OPT | FEAT_COMP, MS_W2)

extern "C" __global__ void __launch_bounds__(WAVE * BIN_WAVES) MS_W2
ms_step_kernel_bins(const BatchDev* __restrict__ batches, const Tile* __restrict__ tiles, const Bin* __restrict__ bins,
                    int n_bins, const TileEnv* __restrict__ tenv, int n_steps) {
    step_bins<0>(batches, tiles, bins, n_bins, tenv, n_steps);
}
extern "C" __global__ void __launch_bounds__(WAVE * BIN_WAVES) MS_W2
ms_step_kernel_bins_opt(const BatchDev* __restrict__ batches, const Tile* __restrict__ tiles, const Bin* __restrict__ bins,
                        int n_bins, const TileEnv* __restrict__ tenv, int n_steps) {
    step_bins<FEAT_OPT>(batches, tiles, bins, n_bins, tenv, n_steps);
}
extern "C" __global__ void __launch_bounds__(WAVE * BIN_WAVES) MS_W2
ms_step_kernel_bins_comp(const BatchDev* __restrict__ batches, const Tile* __restrict__ tiles,
                         const Bin* __restrict__ bins, int n_bins, const TileEnv* __restrict__ tenv, int n_steps) {
    step_bins<FEAT_OPT | FEAT_COMP>(batches, tiles, bins, n_bins, tenv, n_steps);
}

// ============================================================================= reset kernel
// Write the state of the listed envs from a source (the batch's initial state or caller SoA
// arrays of the same shape) and clear their status.  One workgroup per listed env.
extern "C" __global__ void __launch_bounds__(64) ms_reset_kernel(BatchDev bd, const int* __restrict__ env_ids,
                                                               int n_ids, const float* __restrict__ spos,
                                                               const float* __restrict__ squat,
                                                               const float* __restrict__ svel,
                                                               const float* __restrict__ sang) {
    int k = blockIdx.x;
    if (k >= n_ids) return;
    int e = env_ids[k];
    if (e < 0 || e >= bd.E) {
        if (threadIdx.x == 0) atomicAdd(bd.bad_ids, 1);
        return;
    }
    int b0 = bd.body_off[e], b1 = bd.body_off[e + 1];
    const int B = bd.B;
    for (int gi = b0 + int(threadIdx.x); gi < b1; gi += blockDim.x) {
        for (int r = 0; r < 3; ++r) bd.pos[r * B + gi] = spos[r * B + gi];
        for (int r = 0; r < 4; ++r) bd.quat[r * B + gi] = squat[r * B + gi];
        for (int r = 0; r < 3; ++r) bd.vel[r * B + gi] = svel[r * B + gi];
        for (int r = 0; r < 3; ++r) bd.angvel[r * B + gi] = sang[r * B + gi];
        if (bd.forces)
            for (int r = 0; r < 3; ++r) bd.forces[r * B + gi] = 0.0f;
    }
    if (threadIdx.x == 0) {
        bd.status[e] = 0;
        if (bd.cache_hdr) { bd.cache_hdr[2 * e] = 0; bd.cache_hdr[2 * e + 1] = 0; }
    }
}

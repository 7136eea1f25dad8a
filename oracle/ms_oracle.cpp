// ms_oracle.cpp — plain, slow CPU reference of the batched rigid-body step.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU-baseline
// leg load this library.  It shares no code, header or constant table with the GPU library and
// exists to decide what the GPU step must compute.
//
// What it computes.  ManiSkill3 (arXiv 2410.00425) advances thousands of independent,
// heterogeneous scenes with GPU rigid-body simulation (Sec. III-C), tuned by solver position /
// velocity iteration counts (App. E, Setup) and PD joint drives (App. B, Controller).  The paper
// states no contact or solver equations, so this file implements one documented step model,
// each phase named after the published method it restates:
//   S0 frozen step-start quantities; S1 exact AABBs; S2 all-pairs broadphase with filters;
//   S3 narrowphase for sphere / capsule / box / plane pairs (closest points after Ericson,
//      "Real-Time Collision Detection" 5.1.9; separating axes after Gottschalk's OBB test;
//      Sutherland-Hodgman clipping) with a <= 4 point manifold reduction; compound bodies
//      (up to 4 primitive parts, the convex pieces of a decomposed object) by every pair of
//      parts, one manifold per pair of parts with points;
//   S4 contact rows (tangent basis after Duff et al. 2017, "Building an Orthonormal Basis,
//      Revisited"); S4b (optional) cross-step warm start from a contact cache matched by pair
//      and body-frame position; S5 greedy colouring that fixes the Gauss-Seidel order;
//   S6 TGS substeps (sequential impulses with clamped accumulated impulses, warm start across
//      substeps, speculative contacts, Baumgarte bias; patch friction at the manifold centroid
//      with a torsional row; revolute point + 2 angular rows, prismatic rotation lock + 2 rows
//      across the slide axis, each with a per-step Baumgarte rate and extra joint-only passes;
//      one-sided limit rows; PD drive as a soft row after Catto, "Soft Constraints", GDC 2011);
//      symplectic Euler on offsets from the step-start pose;
//   S7 velocity iterations and a restitution pass; S8 write-back with a non-finite guard.
// Templated on float and double.  Built with -ffp-contract=off: no fused multiply-add anywhere.
// Parity pins live in the CPU test suite (closed forms, invariants, brute force).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace orc {

// ----------------------------------------------------------------------------- interface types
// Byte layout of the descriptor records handed over by the input generators (88 / 92 bytes).
struct BodyDesc {
    int32_t shape, flags;
    float dims[3];
    float mass, density, friction, restitution;
    float pos[3], quat[4], linvel[3], angvel[3];
};
struct JointDesc {
    int32_t parent, child;
    float frame_parent[7], frame_child[7];
    float kp, kd, target;
    int32_t type, limited;
    float lower, upper;
};
struct Params {
    float dt;
    int32_t pos_iters, vel_iters, solver;
    float gravity[3];
    float plane_z;
    int32_t plane_enabled;
    float plane_friction, plane_restitution;
    float contact_offset, baumgarte, max_depen_vel, joint_baumgarte, bounce_threshold;
    float lin_damping, ang_damping;
    int32_t max_contacts_per_env;
    int32_t debug_export;
    int32_t joint_iters;
    int32_t max_manifolds_per_env;
    int32_t warm_start;   // != 0: cross-step warm start from the contact cache (S4b)
    float warm_radius;    // matching radius of the cache, m
};
static_assert(sizeof(Params) == 96, "parameter record layout");
static_assert(sizeof(BodyDesc) == 88, "body record layout");
static_assert(sizeof(JointDesc) == 92, "joint record layout");

enum { SPHERE = 0, CAPSULE = 1, BOX = 2, COMPOUND = 3 };
constexpr int MAX_CHILDREN = 4;
// A compound body's parts: up to 4 primitives (sphere / capsule / box) with their poses in the
// body frame (position, then quaternion w, x, y, z).  180 bytes.
struct CompoundDesc {
    int32_t n_children;
    int32_t shape[MAX_CHILDREN];
    float dims[MAX_CHILDREN][3];
    float pose[MAX_CHILDREN][7];
};
static_assert(sizeof(CompoundDesc) == 180, "compound record layout");
enum { STATIC = 1 };
enum { REVOLUTE = 0, PRISMATIC = 1 };
enum { ST_NONFINITE = 1, ST_CONTACT_OVERFLOW = 2, ST_COLOR_OVERFLOW = 4 };
constexpr int PLANE_ID = 0xFFFF;
constexpr int MAX_COLORS = 64;

// ----------------------------------------------------------------------------- small math
template <class T> struct V3 { T x, y, z; };
template <class T> inline V3<T> mk(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> inline V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> inline V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> inline V3<T> operator-(V3<T> a) { return {-a.x, -a.y, -a.z}; }
template <class T> inline V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> inline T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> inline V3<T> cross(V3<T> a, V3<T> b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> inline T len(V3<T> a) { return std::sqrt(dot(a, a)); }
template <class T> inline V3<T> comp(V3<T> a, int i) { (void)a; return i == 0 ? mk<T>(1, 0, 0) : (i == 1 ? mk<T>(0, 1, 0) : mk<T>(0, 0, 1)); }
template <class T> inline T get(V3<T> a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
template <class T> inline void set(V3<T>& a, int i, T v) { if (i == 0) a.x = v; else if (i == 1) a.y = v; else a.z = v; }

template <class T> struct Q { T w, x, y, z; };
template <class T> inline Q<T> qmul(Q<T> a, Q<T> b) {
    return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
            a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
            a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
            a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
template <class T> inline Q<T> qconj(Q<T> a) { return {a.w, -a.x, -a.y, -a.z}; }
template <class T> inline Q<T> qnormalize(Q<T> a) {
    T n = std::sqrt(a.w * a.w + a.x * a.x + a.y * a.y + a.z * a.z);
    T inv = T(1) / n;
    return {a.w * inv, a.x * inv, a.y * inv, a.z * inv};
}

// Row-major 3x3.  Rotation matrix of a unit quaternion, written term by term (the AABB of S1
// depends on these exact operations so that both implementations get identical bits).
template <class T> struct M3 { T m[3][3]; };
template <class T> inline M3<T> rotm(Q<T> q) {
    T xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
    T xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
    T wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z;
    M3<T> r;
    r.m[0][0] = T(1) - T(2) * (yy + zz); r.m[0][1] = T(2) * (xy - wz);        r.m[0][2] = T(2) * (xz + wy);
    r.m[1][0] = T(2) * (xy + wz);        r.m[1][1] = T(1) - T(2) * (xx + zz); r.m[1][2] = T(2) * (yz - wx);
    r.m[2][0] = T(2) * (xz - wy);        r.m[2][1] = T(2) * (yz + wx);        r.m[2][2] = T(1) - T(2) * (xx + yy);
    return r;
}
template <class T> inline V3<T> mul(const M3<T>& a, V3<T> v) {
    return {a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z,
            a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z,
            a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z};
}
template <class T> inline V3<T> mulT(const M3<T>& a, V3<T> v) {
    return {a.m[0][0] * v.x + a.m[1][0] * v.y + a.m[2][0] * v.z,
            a.m[0][1] * v.x + a.m[1][1] * v.y + a.m[2][1] * v.z,
            a.m[0][2] * v.x + a.m[1][2] * v.y + a.m[2][2] * v.z};
}
template <class T> inline V3<T> col(const M3<T>& a, int j) { return {a.m[0][j], a.m[1][j], a.m[2][j]}; }
template <class T> inline V3<T> rotate(Q<T> q, V3<T> v) { return mul(rotm(q), v); }

// Symmetric world inverse inertia R diag(d) R^T (upper triangle computed, then mirrored).
template <class T> inline M3<T> world_inv_inertia(Q<T> q, V3<T> d) {
    M3<T> r = rotm(q), o;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            o.m[i][j] = r.m[i][0] * d.x * r.m[j][0] + r.m[i][1] * d.y * r.m[j][1] + r.m[i][2] * d.z * r.m[j][2];
            o.m[j][i] = o.m[i][j];
        }
    return o;
}

// ----------------------------------------------------------------------------- mass properties
// Uniform density; COM at the shape centre.  Box: m/12 (b^2+c^2, ...) with full sides.  Sphere:
// 2/5 m r^2.  Capsule = cylinder (length L, radius r) + two hemispheres, each hemisphere moved
// from its own centre of mass (3r/8 from its flat face) to the capsule centre (parallel axes).
template <class T> inline T shape_volume(int shape, const T* d) {
    const T pi = T(3.14159265358979323846);
    if (shape == SPHERE) return T(4) / T(3) * pi * d[0] * d[0] * d[0];
    if (shape == CAPSULE) {
        T L = T(2) * d[1];
        return pi * d[0] * d[0] * L + T(4) / T(3) * pi * d[0] * d[0] * d[0];
    }
    return T(8) * d[0] * d[1] * d[2];
}
template <class T> inline V3<T> shape_inertia(int shape, const T* d, T mass) {
    if (shape == SPHERE) { T i = T(2) / T(5) * mass * d[0] * d[0]; return {i, i, i}; }
    if (shape == BOX) {
        T a = T(2) * d[0], b = T(2) * d[1], c = T(2) * d[2];
        return {mass / T(12) * (b * b + c * c), mass / T(12) * (a * a + c * c), mass / T(12) * (a * a + b * b)};
    }
    const T pi = T(3.14159265358979323846);
    T r = d[0], L = T(2) * d[1];
    T vc = pi * r * r * L, vs = T(4) / T(3) * pi * r * r * r;
    T rho = mass / (vc + vs);
    T mc = rho * vc, ms = rho * vs;
    T izz = mc * r * r / T(2) + ms * T(2) * r * r / T(5);
    T ixx = mc * (L * L / T(12) + r * r / T(4)) + ms * (T(2) * r * r / T(5) + L * L / T(4) + T(3) * L * r / T(8));
    return {ixx, ixx, izz};
}

// Compound mass properties (uniform density over the parts; overlapping parts count twice): the
// parts share the mass in proportion to their volumes; each part's inertia about its centre is
// rotated into the body frame, R diag(I) R^T, and moved to the body origin by the parallel-axis
// term m_k (|c|^2 delta_ij - c_i c_j); the parts are summed in order.  The body frame must be
// the principal frame with the centre of mass at its origin (the scene generator builds
// compounds so): only the diagonal is used.
template <class T> struct Compound {
    int n = 0;
    int shape[MAX_CHILDREN] = {0, 0, 0, 0};
    T dims[MAX_CHILDREN][3] = {};
    V3<T> c[MAX_CHILDREN];
    Q<T> q[MAX_CHILDREN];
};
template <class T> inline T compound_volume(const Compound<T>& C) {
    T v = 0;
    for (int k = 0; k < C.n; ++k) v = v + shape_volume<T>(C.shape[k], C.dims[k]);
    return v;
}
template <class T> inline V3<T> compound_inertia(const Compound<T>& C, T mass) {
    const T vt = compound_volume(C);
    T I[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int k = 0; k < C.n; ++k) {
        const T mk_ = mass * (shape_volume<T>(C.shape[k], C.dims[k]) / vt);
        const V3<T> Ik = shape_inertia<T>(C.shape[k], C.dims[k], mk_);
        const M3<T> R = rotm(C.q[k]);
        const T d[3] = {Ik.x, Ik.y, Ik.z};
        const T cc[3] = {C.c[k].x, C.c[k].y, C.c[k].z};
        const T c2 = dot(C.c[k], C.c[k]);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const T rot = R.m[i][0] * d[0] * R.m[j][0] + R.m[i][1] * d[1] * R.m[j][1] + R.m[i][2] * d[2] * R.m[j][2];
                const T par = mk_ * ((i == j ? c2 : T(0)) - cc[i] * cc[j]);
                I[i][j] = I[i][j] + (rot + par);
            }
    }
    return {I[0][0], I[1][1], I[2][2]};
}

// ----------------------------------------------------------------------------- scene storage
template <class T> struct Body {
    int shape = 0, flags = 0;
    int comp = -1;   // compound index (shape COMPOUND)
    T dims[3] = {0, 0, 0};
    T invm = 0;
    V3<T> invI{0, 0, 0};  // body-frame principal inverse inertia
    T mu = 0, e = 0;
    V3<T> x{0, 0, 0};
    Q<T> q{1, 0, 0, 0};
    V3<T> v{0, 0, 0}, w{0, 0, 0};
    bool dyn() const { return !(flags & STATIC); }
};
template <class T> struct Joint {
    int parent, child;
    int type;      // REVOLUTE: rotation about the joint frame's z; PRISMATIC: translation along it
    bool limited;  // position limits [lower, upper] (rad or m)
    V3<T> aA, aB;  // anchors in body frames
    Q<T> QA, QB;   // joint-frame rotations in body frames
    T kp, kd, target;
    T lower, upper;
};

struct PairRec { int32_t env, a, b, npts, decision, kind; double margin, lt1, lt2, ltw, mu, rt; };
struct PointRec { int32_t env, pair; double p[3], n[3], s, ln, ln0; };
struct BlockRec { int32_t env, kind, index, colour; };
// Per-env counters for the work model: candidate pairs per shape pair, points, manifolds, joints,
// colours, dynamic bodies, static bodies.
enum { CNT_PAIRS_TESTED = 0, CNT_CAND = 1, CNT_POINTS = 2, CNT_MANIFOLDS = 3, CNT_COLOURS = 4,
       CNT_DYN = 5, CNT_STATIC = 6, CNT_JOINTS = 7, CNT_KIND0 = 8, N_CNT = 8 + 12 };

// ----------------------------------------------------------------------------- narrowphase
template <class T> struct Pt { V3<T> p, n; T s; };
template <class T> struct Out {
    Pt<T> pt[16];
    int n = 0;
    int decision = 0;
    double margin = 1e30;  // distance of this pair's discrete decisions to their thresholds
    void note(double m) { m = std::fabs(m); if (m < margin) margin = m; }
};

template <class T> struct Shape {
    int type;
    V3<T> c;
    M3<T> R;
    T d[3];
    // capsule segment end points
    V3<T> p0() const { return c - d[1] * col(R, 2); }
    V3<T> p1() const { return c + d[1] * col(R, 2); }
};

// Witness midpoint record: pa on A's surface, pb on B's surface, n from A to B.
template <class T> inline void emit(Out<T>& o, V3<T> pa, V3<T> pb, V3<T> n, T s, T delta) {
    o.note(double(s) - double(delta));
    if (s < delta && o.n < 16) { o.pt[o.n++] = Pt<T>{T(0.5) * (pa + pb), n, s}; }
}

// Closest points of segments P(s) = p1 + s d1 and Q(t) = p2 + t d2, s, t in [0, 1]
// (the clamped-parameter method of Ericson, RTCD 5.1.9, restated).
template <class T> inline void seg_seg(V3<T> p1, V3<T> q1, V3<T> p2, V3<T> q2, T& s, T& t) {
    V3<T> d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
    T a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
    const T eps = T(1e-12);
    auto clamp01 = [](T v) { return v < T(0) ? T(0) : (v > T(1) ? T(1) : v); };
    if (a <= eps && e <= eps) { s = 0; t = 0; return; }
    if (a <= eps) { s = 0; t = clamp01(f / e); return; }
    T c = dot(d1, r);
    if (e <= eps) { t = 0; s = clamp01(-c / a); return; }
    T b = dot(d1, d2);
    T denom = a * e - b * b;
    s = denom != T(0) ? clamp01((b * f - c * e) / denom) : T(0);
    t = (b * s + f) / e;
    if (t < T(0)) { t = 0; s = clamp01(-c / a); }
    else if (t > T(1)) { t = 1; s = clamp01((b - c) / a); }
}
template <class T> inline T closest_on_seg(V3<T> p0, V3<T> p1, V3<T> x) {
    V3<T> d = p1 - p0;
    T dd = dot(d, d);
    if (dd <= T(1e-12)) return T(0);
    T t = dot(x - p0, d) / dd;
    return t < T(0) ? T(0) : (t > T(1) ? T(1) : t);
}

// N4: two spheres; n from A to B (+z when the centres coincide).
template <class T> inline void sphere_sphere(Out<T>& o, V3<T> ca, T ra, V3<T> cb, T rb, T delta) {
    V3<T> d = cb - ca;
    T dist = len(d);
    V3<T> n = dist < T(1e-9) ? mk<T>(0, 0, 1) : (T(1) / dist) * d;
    T s = dist - ra - rb;
    emit(o, ca + ra * n, cb - rb * n, n, s, delta);
}

// Plane (always A, normal +z) against a sphere of centre c.
template <class T> inline void plane_sphere(Out<T>& o, T pz, V3<T> c, T r, T delta) {
    V3<T> n = mk<T>(0, 0, 1);
    T s = c.z - pz - r;
    emit(o, mk<T>(c.x, c.y, pz), c - r * n, n, s, delta);
}

// N2: box corners below plane_z + delta, in corner index order (bit k of the index = + side).
template <class T> inline void plane_box(Out<T>& o, T pz, const Shape<T>& b, T delta) {
    for (int k = 0; k < 8; ++k) {
        V3<T> l = mk<T>((k & 1) ? b.d[0] : -b.d[0], (k & 2) ? b.d[1] : -b.d[1], (k & 4) ? b.d[2] : -b.d[2]);
        V3<T> c = b.c + mul(b.R, l);
        T s = c.z - pz;
        emit(o, mk<T>(c.x, c.y, pz), c, mk<T>(0, 0, 1), s, delta);
    }
}

// N7: box vs sphere, n from the box to the sphere.
template <class T> inline void box_sphere(Out<T>& o, const Shape<T>& bx, V3<T> c, T r, T delta) {
    V3<T> l = mulT(bx.R, c - bx.c);
    V3<T> q = l;
    for (int i = 0; i < 3; ++i) {
        T v = get(l, i), h = bx.d[i];
        set(q, i, v < -h ? -h : (v > h ? h : v));
    }
    V3<T> dl = l - q;
    T d2 = dot(dl, dl);
    if (d2 > T(0)) {
        o.decision = 0;
        T dist = std::sqrt(d2);
        V3<T> n = mul(bx.R, (T(1) / dist) * dl);
        emit(o, bx.c + mul(bx.R, q), c - r * n, n, dist - r, delta);
        o.note(double(dist));
    } else {
        // centre inside: least-penetration face (lowest axis on ties)
        int best = 0;
        T bd = bx.d[0] - std::fabs(l.x);
        for (int i = 1; i < 3; ++i) {
            T di = bx.d[i] - std::fabs(get(l, i));
            if (di < bd) { o.note(double(bd) - double(di)); bd = di; best = i; }
            else o.note(double(di) - double(bd));
        }
        T sg = get(l, best) >= T(0) ? T(1) : T(-1);
        V3<T> nl = mk<T>(0, 0, 0);
        set(nl, best, sg);
        V3<T> n = mul(bx.R, nl);
        V3<T> face = l;
        set(face, best, sg * bx.d[best]);
        o.decision = 1 + best;
        emit(o, bx.c + mul(bx.R, face), c - r * n, n, -bd - r, delta);
    }
}

// Shapes' support half-width along unit axis L.
template <class T> inline T box_extent(const Shape<T>& b, V3<T> L) {
    return (b.d[0] * std::fabs(dot(col(b.R, 0), L)) + b.d[1] * std::fabs(dot(col(b.R, 1), L))) +
           b.d[2] * std::fabs(dot(col(b.R, 2), L));
}
template <class T> inline T tie_tol(T s, T hmin) { return T(0.05) * std::fabs(s) + T(0.01) * hmin; }

// Clip the parameter interval [t0, t1] of segment p0 + t (p1 - p0) to the slab |(x - c).a| <= h.
template <class T> inline void clip_slab(V3<T> p0, V3<T> p1, V3<T> c, V3<T> a, T h, T& t0, T& t1) {
    T u0 = dot(p0 - c, a), du = dot(p1 - p0, a);
    if (std::fabs(du) < T(1e-12)) {
        if (u0 > h || u0 < -h) { t0 = T(1); t1 = T(0); }
        return;
    }
    T ta = (-h - u0) / du, tb = (h - u0) / du;
    if (ta > tb) std::swap(ta, tb);
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
}

// N8: box vs capsule, n from the box to the capsule.  Separating axes: the 3 box face normals,
// then axis x box edge for the 3 edge directions.  Face axes are preferred; an edge axis wins
// only when its separation exceeds the best face's by more than the tie tolerance.
template <class T> inline void box_capsule(Out<T>& o, const Shape<T>& bx, const Shape<T>& cp, T delta) {
    V3<T> P0 = cp.p0(), P1 = cp.p1(), u = col(cp.R, 2);
    T rc = cp.d[0], hl = cp.d[1];
    V3<T> dc = cp.c - bx.c;
    T sep[6];
    V3<T> ax[6];
    bool valid[6];
    for (int i = 0; i < 3; ++i) {
        V3<T> L = col(bx.R, i);
        if (dot(L, dc) < T(0)) L = -L;
        ax[i] = L; valid[i] = true;
        sep[i] = dot(dc, L) - hl * std::fabs(dot(u, L)) - bx.d[i] - rc;
    }
    for (int i = 0; i < 3; ++i) {
        V3<T> L = cross(u, col(bx.R, i));
        T l = len(L);
        valid[3 + i] = l >= T(1e-6);
        if (!valid[3 + i]) { sep[3 + i] = T(-1e30); ax[3 + i] = mk<T>(0, 0, 0); continue; }
        L = (T(1) / l) * L;
        if (dot(L, dc) < T(0)) L = -L;
        ax[3 + i] = L;
        sep[3 + i] = dot(dc, L) - hl * std::fabs(dot(u, L)) - box_extent(bx, L) - rc;
    }
    T hmin = std::min(std::min(bx.d[0], bx.d[1]), std::min(bx.d[2], rc));
    int bf = 0;
    for (int i = 1; i < 3; ++i) { o.note(double(sep[i]) - double(sep[bf])); if (sep[i] > sep[bf]) bf = i; }
    int be = -1;
    for (int i = 3; i < 6; ++i)
        if (valid[i]) { if (be >= 0) o.note(double(sep[i]) - double(sep[be])); if (be < 0 || sep[i] > sep[be]) be = i; }
    int best = bf;
    if (be >= 0) {
        T thr = sep[bf] + tie_tol(sep[bf], hmin);
        o.note(double(sep[be]) - double(thr));
        if (sep[be] > thr) best = be;
    }
    T smax = sep[0];
    for (int i = 1; i < 6; ++i) if (valid[i] && sep[i] > smax) smax = sep[i];
    o.note(double(smax) - double(delta));
    o.decision = best;
    if (smax >= delta) return;
    if (best < 3) {
        int i = best;
        V3<T> nr = ax[i];
        int j1 = (i + 1) % 3, j2 = (i + 2) % 3;
        T t0 = 0, t1 = 1;
        clip_slab(P0, P1, bx.c, col(bx.R, j1), bx.d[j1], t0, t1);
        clip_slab(P0, P1, bx.c, col(bx.R, j2), bx.d[j2], t0, t1);
        o.note(double(t1) - double(t0));
        if (t0 <= t1) {
            T ts[2] = {t0, t1};
            int np = t1 > t0 ? 2 : 1;
            for (int k = 0; k < np; ++k) {
                V3<T> C = P0 + ts[k] * (P1 - P0);
                T above = dot(C - bx.c, nr) - bx.d[i];
                emit(o, C - above * nr, C - rc * nr, nr, above - rc, delta);
            }
        } else {
            // Segment outside the face's prism: nearest of the face's 4 boundary edges.
            o.decision = 6 + i;
            T bestd = T(1e30);
            V3<T> bs{0, 0, 0}, be2{0, 0, 0};
            V3<T> fc = bx.c + bx.d[i] * nr;
            for (int k = 0; k < 4; ++k) {
                int along = (k < 2) ? j1 : j2, other = (k < 2) ? j2 : j1;
                T sg = (k & 1) ? T(1) : T(-1);
                V3<T> ec = fc + (sg * bx.d[other]) * col(bx.R, other);
                V3<T> e0 = ec - bx.d[along] * col(bx.R, along), e1 = ec + bx.d[along] * col(bx.R, along);
                T s, t;
                seg_seg(P0, P1, e0, e1, s, t);
                V3<T> cs = P0 + s * (P1 - P0), ce = e0 + t * (e1 - e0);
                V3<T> dd = cs - ce;
                T d2 = dot(dd, dd);
                if (k > 0) o.note(double(d2) - double(bestd));
                if (d2 < bestd) { bestd = d2; bs = cs; be2 = ce; }
            }
            T dist = std::sqrt(bestd);
            V3<T> n = dist > T(1e-9) ? (T(1) / dist) * (bs - be2) : nr;
            emit(o, be2, bs - rc * n, n, dist - rc, delta);
        }
    } else {
        int i = best - 3;
        V3<T> L = ax[best];
        V3<T> ec = bx.c;
        for (int j = 0; j < 3; ++j) {
            if (j == i) continue;
            T dj = dot(col(bx.R, j), L);
            o.note(double(dj));
            ec = ec + ((dj >= T(0) ? T(1) : T(-1)) * bx.d[j]) * col(bx.R, j);
        }
        V3<T> e0 = ec - bx.d[i] * col(bx.R, i), e1 = ec + bx.d[i] * col(bx.R, i);
        T s, t;
        seg_seg(P0, P1, e0, e1, s, t);
        V3<T> cs = P0 + s * (P1 - P0), ce = e0 + t * (e1 - e0);
        T sp = dot(cs - ce, L) - rc;
        emit(o, ce, cs - rc * L, L, sp, delta);
    }
}

// Sutherland-Hodgman: keep the part of polygon `in` with dot(x, a) <= off (at most 8 vertices).
template <class T> inline int clip_poly(const V3<T>* in, int n, V3<T> a, T off, V3<T>* out) {
    int m = 0;
    for (int k = 0; k < n; ++k) {
        V3<T> p = in[k], q = in[(k + 1) % n];
        T dp = dot(p, a) - off, dq = dot(q, a) - off;
        if (dp <= T(0) && m < 8) out[m++] = p;
        if (((dp < T(0) && dq > T(0)) || (dp > T(0) && dq < T(0))) && m < 8) {
            T t = dp / (dp - dq);
            out[m++] = p + t * (q - p);
        }
    }
    return m;
}

// N9: box vs box, n from A to B.  15 separating axes (A faces, B faces, 9 edge crosses).
template <class T> inline void box_box(Out<T>& o, const Shape<T>& A, const Shape<T>& B, T delta) {
    V3<T> d = B.c - A.c;
    T sep[15];
    V3<T> ax[15];
    bool valid[15];
    for (int k = 0; k < 15; ++k) {
        V3<T> L;
        if (k < 3) L = col(A.R, k);
        else if (k < 6) L = col(B.R, k - 3);
        else {
            L = cross(col(A.R, (k - 6) / 3), col(B.R, (k - 6) % 3));
            T l = len(L);
            if (l < T(1e-6)) { valid[k] = false; sep[k] = T(-1e30); ax[k] = mk<T>(0, 0, 0); continue; }
            L = (T(1) / l) * L;
        }
        if (dot(L, d) < T(0)) L = -L;
        valid[k] = true;
        ax[k] = L;
        sep[k] = dot(d, L) - box_extent(A, L) - box_extent(B, L);
    }
    T hmin = std::min(std::min(std::min(A.d[0], A.d[1]), std::min(A.d[2], B.d[0])), std::min(B.d[1], B.d[2]));
    int fa = 0, fb = 3, fe = -1;
    for (int k = 1; k < 3; ++k) { o.note(double(sep[k]) - double(sep[fa])); if (sep[k] > sep[fa]) fa = k; }
    for (int k = 4; k < 6; ++k) { o.note(double(sep[k]) - double(sep[fb])); if (sep[k] > sep[fb]) fb = k; }
    for (int k = 6; k < 15; ++k)
        if (valid[k]) { if (fe >= 0) o.note(double(sep[k]) - double(sep[fe])); if (fe < 0 || sep[k] > sep[fe]) fe = k; }
    int best = fb;
    {
        T thr = sep[fb] + tie_tol(sep[fb], hmin);
        o.note(double(sep[fa]) - double(thr));
        if (sep[fa] > thr) best = fa;
    }
    if (fe >= 0) {
        T thr = sep[best] + tie_tol(sep[best], hmin);
        o.note(double(sep[fe]) - double(thr));
        if (sep[fe] > thr) best = fe;
    }
    T smax = sep[0];
    for (int k = 1; k < 15; ++k) if (valid[k] && sep[k] > smax) smax = sep[k];
    o.note(double(smax) - double(delta));
    o.decision = best;
    if (smax >= delta) return;

    if (best < 6) {
        bool refA = best < 3;
        const Shape<T>& Rf = refA ? A : B;
        const Shape<T>& In = refA ? B : A;
        int ri = refA ? best : best - 3;
        V3<T> nref = refA ? ax[best] : -ax[best];  // outward normal of the reference face, toward In
        // incident face: most anti-parallel to nref (lowest axis on ties)
        int ii = 0;
        T bd = std::fabs(dot(col(In.R, 0), nref));
        for (int j = 1; j < 3; ++j) {
            T dj = std::fabs(dot(col(In.R, j), nref));
            o.note(double(dj) - double(bd));
            if (dj > bd) { bd = dj; ii = j; }
        }
        T sgn = dot(col(In.R, ii), nref) >= T(0) ? T(-1) : T(1);
        V3<T> fcen = In.c + (sgn * In.d[ii]) * col(In.R, ii);
        int u = (ii + 1) % 3, v = (ii + 2) % 3;
        V3<T> U = In.d[u] * col(In.R, u), W = In.d[v] * col(In.R, v);
        V3<T> poly[16], tmp[16];
        poly[0] = fcen + U + W; poly[1] = fcen - U + W; poly[2] = fcen - U - W; poly[3] = fcen + U - W;
        int n = 4;
        int r1 = (ri + 1) % 3, r2 = (ri + 2) % 3;
        V3<T> a1 = col(Rf.R, r1), a2 = col(Rf.R, r2);
        n = clip_poly(poly, n, a1, dot(Rf.c, a1) + Rf.d[r1], tmp);
        n = clip_poly(tmp, n, -a1, -dot(Rf.c, a1) + Rf.d[r1], poly);
        n = clip_poly(poly, n, a2, dot(Rf.c, a2) + Rf.d[r2], tmp);
        n = clip_poly(tmp, n, -a2, -dot(Rf.c, a2) + Rf.d[r2], poly);
        V3<T> nAB = refA ? nref : -nref;
        for (int k = 0; k < n; ++k) {
            V3<T> p = poly[k];
            T s = dot(p - Rf.c, nref) - Rf.d[ri];
            V3<T> onref = p - s * nref;
            if (refA) emit(o, onref, p, nAB, s, delta);
            else emit(o, p, onref, nAB, s, delta);
        }
    } else {
        int ia = (best - 6) / 3, ib = (best - 6) % 3;
        V3<T> L = ax[best];
        V3<T> ca = A.c, cb = B.c;
        for (int j = 0; j < 3; ++j) {
            if (j != ia) { T dj = dot(col(A.R, j), L); o.note(double(dj)); ca = ca + ((dj >= T(0) ? T(1) : T(-1)) * A.d[j]) * col(A.R, j); }
            if (j != ib) { T dj = dot(col(B.R, j), L); o.note(double(dj)); cb = cb + ((dj >= T(0) ? T(-1) : T(1)) * B.d[j]) * col(B.R, j); }
        }
        V3<T> a0 = ca - A.d[ia] * col(A.R, ia), a1 = ca + A.d[ia] * col(A.R, ia);
        V3<T> b0 = cb - B.d[ib] * col(B.R, ib), b1 = cb + B.d[ib] * col(B.R, ib);
        T s, t;
        seg_seg(a0, a1, b0, b1, s, t);
        V3<T> pa = a0 + s * (a1 - a0), pb = b0 + t * (b1 - b0);
        emit(o, pa, pb, L, dot(pb - pa, L), delta);
    }
}

// N6: capsule vs capsule, n from A to B.
template <class T> inline void capsule_capsule(Out<T>& o, const Shape<T>& A, const Shape<T>& B, T delta) {
    V3<T> a0 = A.p0(), a1 = A.p1(), b0 = B.p0(), b1 = B.p1();
    V3<T> d1 = a1 - a0, d2 = b1 - b0;
    V3<T> cr = cross(d1, d2);
    T lhs = dot(cr, cr), rhs = T(1e-6) * dot(d1, d1) * dot(d2, d2);
    o.note(double(lhs) - double(rhs));
    if (lhs < rhs) {
        // parallel: the overlap of B's projection onto A's segment gives two points
        T dd = dot(d1, d1);
        T s0 = dot(b0 - a0, d1) / dd, s1 = dot(b1 - a0, d1) / dd;
        T lo = std::max(T(0), std::min(s0, s1)), hi = std::min(T(1), std::max(s0, s1));
        o.note(double(hi) - double(lo));
        if (lo < hi) {
            o.decision = 1;
            T ss[2] = {lo, hi};
            for (int k = 0; k < 2; ++k) {
                V3<T> pa = a0 + ss[k] * d1;
                T t = closest_on_seg(b0, b1, pa);
                sphere_sphere(o, pa, A.d[0], b0 + t * d2, B.d[0], delta);
            }
            return;
        }
    }
    o.decision = 0;
    T s, t;
    seg_seg(a0, a1, b0, b1, s, t);
    sphere_sphere(o, a0 + s * d1, A.d[0], b0 + t * d2, B.d[0], delta);
}

template <class T> inline void flip(Out<T>& o, int from) {
    for (int k = from; k < o.n; ++k) o.pt[k].n = -o.pt[k].n;
}

// Type dispatch for two bodies (A = lower index).  kind = 3 * min(shape) + max(shape) style code.
template <class T> inline void narrow(Out<T>& o, const Shape<T>& A, const Shape<T>& B, T delta) {
    int ta = A.type, tb = B.type;
    if (ta == SPHERE && tb == SPHERE) { sphere_sphere(o, A.c, A.d[0], B.c, B.d[0], delta); return; }
    if (ta == SPHERE && tb == CAPSULE) {
        T t = closest_on_seg(B.p0(), B.p1(), A.c);
        sphere_sphere(o, A.c, A.d[0], B.p0() + t * (B.p1() - B.p0()), B.d[0], delta);
        return;
    }
    if (ta == CAPSULE && tb == SPHERE) {
        T t = closest_on_seg(A.p0(), A.p1(), B.c);
        sphere_sphere(o, A.p0() + t * (A.p1() - A.p0()), A.d[0], B.c, B.d[0], delta);
        return;
    }
    if (ta == CAPSULE && tb == CAPSULE) { capsule_capsule(o, A, B, delta); return; }
    if (ta == BOX && tb == SPHERE) { box_sphere(o, A, B.c, B.d[0], delta); return; }
    if (ta == SPHERE && tb == BOX) { box_sphere(o, B, A.c, A.d[0], delta); flip(o, 0); return; }
    if (ta == BOX && tb == CAPSULE) { box_capsule(o, A, B, delta); return; }
    if (ta == CAPSULE && tb == BOX) { box_capsule(o, B, A, delta); flip(o, 0); return; }
    box_box(o, A, B, delta);
}

template <class T> inline void narrow_plane(Out<T>& o, T pz, const Shape<T>& B, T delta) {
    if (B.type == SPHERE) plane_sphere(o, pz, B.c, B.d[0], delta);
    else if (B.type == CAPSULE) { plane_sphere(o, pz, B.p0(), B.d[0], delta); plane_sphere(o, pz, B.p1(), B.d[0], delta); }
    else plane_box(o, pz, B, delta);
}

// Manifold reduction to at most 4 points: deepest; farthest from it; largest triangle; the point
// adding the most area outside the triangle.  Lowest index wins every tie.  Kept points stay in
// their original order.
template <class T> inline void reduce4(Out<T>& o, int* picked = nullptr) {
    if (o.n <= 4) return;
    int n = o.n;
    bool used[16] = {false};
    int k0 = 0;
    for (int k = 1; k < n; ++k) { o.note(double(o.pt[k].s) - double(o.pt[k0].s)); if (o.pt[k].s < o.pt[k0].s) k0 = k; }
    used[k0] = true;
    // each selection starts from the first unused point, so an index is always valid
    int k1 = -1; T b1 = T(-1);
    for (int k = 0; k < n; ++k) {
        if (used[k]) continue;
        V3<T> d = o.pt[k].p - o.pt[k0].p;
        T v = dot(d, d);
        if (k1 >= 0) o.note(double(v) - double(b1));
        if (k1 < 0 || v > b1) { b1 = v; k1 = k; }
    }
    used[k1] = true;
    int k2 = -1; T b2 = T(-1);
    V3<T> e01 = o.pt[k1].p - o.pt[k0].p;
    for (int k = 0; k < n; ++k) {
        if (used[k]) continue;
        V3<T> c = cross(e01, o.pt[k].p - o.pt[k0].p);
        T v = dot(c, c);
        if (k2 >= 0) o.note(double(v) - double(b2));
        if (k2 < 0 || v > b2) { b2 = v; k2 = k; }
    }
    used[k2] = true;
    V3<T> nt = cross(e01, o.pt[k2].p - o.pt[k0].p);
    int tri[3] = {k0, k1, k2};
    int k3 = -1; T b3 = T(-1e30);
    for (int k = 0; k < n; ++k) {
        if (used[k]) continue;
        T best = T(-1e30);
        for (int e = 0; e < 3; ++e) {
            V3<T> pa = o.pt[tri[e]].p, pb = o.pt[tri[(e + 1) % 3]].p;
            T v = -dot(cross(pb - pa, o.pt[k].p - pa), nt);
            if (v > best) best = v;
        }
        if (k3 >= 0) o.note(double(best) - double(b3));
        if (k3 < 0 || best > b3) { b3 = best; k3 = k; }
    }
    used[k3] = true;
    if (picked) { picked[0] = k0; picked[1] = k1; picked[2] = k2; picked[3] = k3; }
    int m = 0;
    for (int k = 0; k < n; ++k) if (used[k]) o.pt[m++] = o.pt[k];
    o.n = m;
}

// ----------------------------------------------------------------------------- solver rows
// One contact point: the normal row.
template <class T> struct CRow {
    int a, b;  // body indices, -1 = plane/world
    V3<T> rA, rB, n;
    T mn, s0, e, vnpre;
    T ln;
    T ln0;     // the impulse the step started from (cross-step warm start; 0 otherwise), for the record
};
// One manifold: its points' normal rows plus the friction patch at the points' centroid (two
// tangent rows bounded by mu times the summed normal impulse, and a torsional row about the
// mean normal bounded by mu times the mean point radius times the summed normal impulse).
template <class T> struct Manifold {
    int a, b, first, count, colour, pair;
    int part;   // pair of parts of a compound body pair (0 for primitive pairs)
    V3<T> base, offB;  // frame of the contact geometry (for the record)
    V3<T> rA, rB, nb, t1, t2;
    T mt1, mt2, mtw, mu, rt;
    T lt1, lt2, ltw;
};
// Accumulated joint impulses of a step: revolute lp = point block, la[0..1] = angular block;
// prismatic lp[0..1] = the two rows across the slide axis, la[0..2] = the rotation lock; ld =
// drive; ll = lower and upper limit rows.
template <class T> struct JState { T lp[3], la[3], ld, ll[2]; };

// Contact cache of the cross-step warm start (S4b): the last step's manifolds in canonical order,
// each with its pair key, the tangential impulse of its friction patch as a world vector, its
// twist impulse and its points, and per point the contact position in body B's frame at that
// step's start and the final normal impulse.
template <class T> struct CacheMan { int key, first, count; V3<T> pt; T ltw; };
template <class T> struct CachePt { V3<T> rl; T ln; };

template <class T> struct Env {
    const std::vector<Compound<T>>* comps = nullptr;   // the batch's compound table
    std::vector<Body<T>> bodies;
    std::vector<Joint<T>> joints;
    int status = 0;
    std::vector<V3<T>> force;  // net contact force on each body, averaged over the last step
    std::vector<CacheMan<T>> cman;
    std::vector<CachePt<T>> cpt;
};

template <class T> struct StepCtx {
    const Params* P;
    T delta, plane_z;
    bool plane;
    T plane_mu, plane_e;
};

template <class T> struct BodyView {
    T invm;
    M3<T> Iw;  // world inverse inertia, frozen for the step
};

// Half size along world axis r of a primitive with rotation R: add, multiply and abs only.
template <class T> inline T part_half(int shape, const T* d, const M3<T>& R, int r) {
    if (shape == BOX) return (std::fabs(R.m[r][0]) * d[0] + std::fabs(R.m[r][1]) * d[1]) + std::fabs(R.m[r][2]) * d[2];
    if (shape == SPHERE) return d[0];
    return std::fabs(R.m[r][2]) * d[1] + d[0];
}

template <class T> inline V3<T> vel_at(const Body<T>* b, V3<T> r) {
    if (!b) return mk<T>(0, 0, 0);
    return b->v + cross(b->w, r);
}

// atan(t) for t in [0, 1]: two half-angle reductions, tan(a/2) = t / (1 + sqrt(1 + t^2)), bring
// the argument below tan(pi/16) ~ 0.2; the alternating Taylor series to u^15 then has a
// truncation error below 1e-13; the angle is scaled back by 4.
template <class T> inline T atan_unit(T t) {
    T u = t / (T(1) + std::sqrt(T(1) + t * t));
    u = u / (T(1) + std::sqrt(T(1) + u * u));
    T u2 = u * u;
    T p = T(1) / T(15);
    p = T(1) / T(13) - u2 * p;
    p = T(1) / T(11) - u2 * p;
    p = T(1) / T(9) - u2 * p;
    p = T(1) / T(7) - u2 * p;
    p = T(1) / T(5) - u2 * p;
    p = T(1) / T(3) - u2 * p;
    p = T(1) - u2 * p;
    return T(4) * (u * p);
}
// atan2(y, x) for x >= 0 (result in [-pi/2, pi/2]) from atan_unit and the reflection
// atan(t) = pi/2 - atan(1/t).
template <class T> inline T atan2_pos(T y, T x) {
    T ay = std::fabs(y);
    T a;
    if (ay <= x) a = x > T(0) ? atan_unit(ay / x) : T(0);
    else a = T(3.14159265358979323846) / T(2) - atan_unit(x / ay);
    return y < T(0) ? -a : a;
}

// Duff et al. 2017 branchless orthonormal basis of unit n: returns t1 (t2 = n x t1).
template <class T> inline V3<T> onb_t1(V3<T> n) {
    T sg = std::copysign(T(1), n.z);
    T a = T(-1) / (sg + n.z);
    T b = n.x * n.y * a;
    return mk<T>(T(1) + sg * n.x * n.x * a, sg * b, -sg * n.x);
}

// ----------------------------------------------------------------------------- random draws
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11): ten rounds of the multiply-xor bijection on a 4 x 32-bit counter, the 2 x 32-bit key
// bumped by the Weyl constants between rounds.
inline void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = uint64_t(0xD2511F53u) * c0, p1 = uint64_t(0xCD9E8D57u) * c2;
        const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0, n2 = uint32_t(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = uint32_t(p1); c2 = n2; c3 = uint32_t(p0);
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
// A uniform in [0, 1) from the top 24 bits of a draw (exact in float and double).
template <class T> inline T unit24(uint32_t x) { return T(x >> 8) * T(5.9604644775390625e-08); }

// Reset draws of one env: stream (env, reset_count, purpose, index) under key = the seed.
struct ResetStream {
    uint32_t key[2], env, count;
    void draw(uint32_t purpose, uint32_t index, uint32_t out[4]) const {
        const uint32_t ctr[4] = {env, count, purpose, index};
        philox4x32_10(ctr, key, out);
    }
};
// A standard normal deviate approximated by the sum of 12 uniforms minus 6 (the Irwin-Hall
// construction: mean 0, variance 1), from three consecutive blocks; summed in draw order.
template <class T> inline T normal12(const ResetStream& rs, uint32_t purpose, uint32_t first_block) {
    T sum = 0;
    for (uint32_t b = 0; b < 3; ++b) {
        uint32_t u[4];
        rs.draw(purpose, first_block + b, u);
        for (int k = 0; k < 4; ++k) sum = sum + unit24<T>(u[k]);
    }
    return sum - T(6);
}
// sin and cos of x in [-pi/2 - 0.2, pi/2 + 0.2] by their Taylor series to x^17 / x^18 (Horner in
// x^2; truncation below 1e-11), from correctly rounded operations only.
template <class T> inline T sin_series(T x) {
    const T x2 = x * x;
    T p = T(1) / T(355687428096000.0);                // 1 / 17!
    p = T(-1) / T(1307674368000.0) + x2 * p;          // 1 / 15!
    p = T(1) / T(6227020800.0) + x2 * p;              // 1 / 13!
    p = T(-1) / T(39916800.0) + x2 * p;               // 1 / 11!
    p = T(1) / T(362880.0) + x2 * p;                  // 1 / 9!
    p = T(-1) / T(5040.0) + x2 * p;                   // 1 / 7!
    p = T(1) / T(120.0) + x2 * p;                     // 1 / 5!
    p = T(-1) / T(6.0) + x2 * p;                      // 1 / 3!
    p = T(1) + x2 * p;
    return x * p;
}
template <class T> inline T cos_series(T x) {
    const T x2 = x * x;
    T p = T(-1) / T(6402373705728000.0);              // 1 / 18!
    p = T(1) / T(20922789888000.0) + x2 * p;          // 1 / 16!
    p = T(-1) / T(87178291200.0) + x2 * p;            // 1 / 14!
    p = T(1) / T(479001600.0) + x2 * p;               // 1 / 12!
    p = T(-1) / T(3628800.0) + x2 * p;                // 1 / 10!
    p = T(1) / T(40320.0) + x2 * p;                   // 1 / 8!
    p = T(-1) / T(720.0) + x2 * p;                    // 1 / 6!
    p = T(1) / T(24.0) + x2 * p;                      // 1 / 4!
    p = T(-1) / T(2.0) + x2 * p;                      // 1 / 2!
    return T(1) + x2 * p;
}

// Result of one env step for the test record.
struct EnvRecord {
    std::vector<PairRec> pairs;
    std::vector<PointRec> points;
    std::vector<BlockRec> blocks;
    int64_t cnt[N_CNT];
    double min_margin;
};

template <class T> struct Stepper {
    const Params& P;
    Env<T>& E;
    EnvRecord* rec;
    int env_id;
    // per-step working state
    std::vector<BodyView<T>> bv;
    std::vector<V3<T>> x0, dx;  // step-start centre and its offset accumulated over substeps
    std::vector<Q<T>> q0, dq;   // step-start orientation and the rotation accumulated since
    std::vector<CRow<T>> rows;
    std::vector<Manifold<T>> mans;
    std::vector<JState<T>> js;
    int ncol = 0;
    std::vector<std::pair<int, int>> order;  // (colour, block id) solve order
    T h = 0;

    Stepper(const Params& p, Env<T>& e, EnvRecord* r, int id) : P(p), E(e), rec(r), env_id(id) {}

    T invm(int i) const { return i < 0 ? T(0) : bv[i].invm; }
    M3<T> Iw(int i) const { if (i < 0) { M3<T> z{}; return z; } return bv[i].Iw; }
    bool dyn(int i) const { return i >= 0 && E.bodies[i].dyn(); }

    Shape<T> shape_of(int i) const {
        const Body<T>& b = E.bodies[i];
        Shape<T> s;
        s.type = b.shape;
        s.c = b.x;
        s.R = rotm(b.q);
        s.d[0] = b.dims[0]; s.d[1] = b.dims[1]; s.d[2] = b.dims[2];
        return s;
    }

    // Apply an impulse P (world) at arms rA, rB: -P on A, +P on B.
    void apply(int a, int b, V3<T> rA, V3<T> rB, V3<T> Pv) {
        if (dyn(a)) {
            Body<T>& A = E.bodies[a];
            A.v = A.v - invm(a) * Pv;
            A.w = A.w - mul(bv[a].Iw, cross(rA, Pv));
        }
        if (dyn(b)) {
            Body<T>& B = E.bodies[b];
            B.v = B.v + invm(b) * Pv;
            B.w = B.w + mul(bv[b].Iw, cross(rB, Pv));
        }
    }
    void apply_ang(int a, int b, V3<T> Lv) {
        if (dyn(a)) E.bodies[a].w = E.bodies[a].w - mul(bv[a].Iw, Lv);
        if (dyn(b)) E.bodies[b].w = E.bodies[b].w + mul(bv[b].Iw, Lv);
    }
    T eff(int a, int b, V3<T> rA, V3<T> rB, V3<T> x) const {
        T k = invm(a) + invm(b);
        if (a >= 0) { V3<T> c = cross(rA, x); k = k + dot(c, mul(bv[a].Iw, c)); }
        if (b >= 0) { V3<T> c = cross(rB, x); k = k + dot(c, mul(bv[b].Iw, c)); }
        return k > T(0) ? T(1) / k : T(0);
    }

    // ------------------------------------------------------------- S0..S5: detection and rows
    // ------------------------------------------------------------- S4b cross-step warm start
    // Key of a manifold, increasing in canonical order: (lower body, partner, pair of parts), the
    // ground plane after every partner of its body.
    static int man_key(const Manifold<T>& m) {
        return ((m.a >= 0 ? (m.a << 8) | m.b : (m.b << 8) | 0xFF) << 4) | m.part;
    }
    // Initial impulses from the last step's cache: a manifold whose pair is cached takes, for each
    // of its points, the normal impulse of the nearest cached point of that pair (positions in
    // body B's frame at the step start, squared distance below warm_radius^2, the first cached
    // point on ties, none beyond the radius), and the cached tangential impulse vector projected
    // on its new tangents t1, t2, and the cached twist impulse.
    void warm_from_cache() {
        const T r2 = T(P.warm_radius) * T(P.warm_radius);
        const int nc = int(E.cman.size());
        for (Manifold<T>& M : mans) {
            const int key = man_key(M);
            int lo = 0, hi = nc;
            while (lo < hi) {
                const int mid = (lo + hi) / 2;
                if (E.cman[mid].key < key) lo = mid + 1; else hi = mid;
            }
            if (lo == nc || E.cman[lo].key != key) continue;
            const CacheMan<T>& C = E.cman[lo];
            const M3<T> RB = rotm(q0[M.b]);
            for (int k = 0; k < M.count; ++k) {
                CRow<T>& r = rows[M.first + k];
                const V3<T> rl = mulT(RB, r.rB);
                T best = r2;
                int bj = -1;
                for (int j = 0; j < C.count; ++j) {
                    const V3<T> d = rl - E.cpt[C.first + j].rl;
                    const T d2 = dot(d, d);
                    if (d2 < best) { best = d2; bj = j; }
                }
                if (bj >= 0) r.ln = E.cpt[C.first + bj].ln;
                r.ln0 = r.ln;
            }
            M.lt1 = dot(C.pt, M.t1);
            M.lt2 = dot(C.pt, M.t2);
            M.ltw = C.ltw;
        }
    }
    // The cache for the next step: every manifold and point of this step with its final impulses.
    void write_cache() {
        E.cman.clear();
        E.cpt.clear();
        for (const Manifold<T>& M : mans) {
            CacheMan<T> C;
            C.key = man_key(M);
            C.first = int(E.cpt.size());
            C.count = M.count;
            C.pt = M.lt1 * M.t1 + M.lt2 * M.t2;
            C.ltw = M.ltw;
            E.cman.push_back(C);
            const M3<T> RB = rotm(q0[M.b]);
            for (int k = 0; k < M.count; ++k) {
                const CRow<T>& r = rows[M.first + k];
                E.cpt.push_back(CachePt<T>{mulT(RB, r.rB), r.ln});
            }
        }
    }

    // ------------------------------------------------------------- compound pairs
    // The primitive parts of body i with its centre at `cen` (pair frame): the body itself, or
    // each part of a compound at cen + R c_k with rotation R(q q_k).
    int parts(int i, V3<T> cen, Shape<T>* out) const {
        const Body<T>& b = E.bodies[i];
        if (b.shape != COMPOUND) {
            out[0] = shape_of(i);
            out[0].c = cen;
            return 1;
        }
        const Compound<T>& C = (*E.comps)[b.comp];
        const M3<T> R = rotm(b.q);
        for (int k = 0; k < C.n; ++k) {
            out[k].type = C.shape[k];
            out[k].c = cen + mul(R, C.c[k]);
            out[k].R = rotm(qmul(b.q, C.q[k]));
            out[k].d[0] = C.dims[k][0]; out[k].d[1] = C.dims[k][1]; out[k].d[2] = C.dims[k][2];
        }
        return C.n;
    }
    // The midphase of compound pairs, in the pair frame: boxes of two parts grown by the contact
    // offset overlap on every axis, or a part's grown box reaches the ground at z = 0 (add,
    // subtract, multiply, abs and compare only, as in the broadphase).
    static bool part_boxes_meet(const Shape<T>& A, const Shape<T>& B, T delta) {
        for (int r = 0; r < 3; ++r) {
            const T ha = part_half(A.type, A.d, A.R, r) + delta, hb = part_half(B.type, B.d, B.R, r) + delta;
            const T ca = get(A.c, r), cb = get(B.c, r);
            if (!(ca - ha <= cb + hb && cb - hb <= ca + ha)) return false;
        }
        return true;
    }
    static bool part_box_reaches_plane(const Shape<T>& B, T delta) {
        return B.c.z - (part_half(B.type, B.d, B.R, 2) + delta) <= T(0);
    }

    // Contact points of a pair with a compound body (a = -1: the ground plane; B's centre at cB):
    // every pair of parts, A's parts outer, whose boxes meet (the broadphase's rule at the level
    // of parts: boxes grown by the contact offset overlap, or reach the ground), through the
    // primitive narrowphase, each reduced to at most 4 points: one point set per pair of parts,
    // each becoming its own manifold (its own friction patch: parts of one compound may touch a
    // body from opposite sides).  Returns the number of part pairs; the decision code (in o[0])
    // is 64 + the index of the first part pair that produced points (63: none) and the margin
    // the smallest over the tested pairs; every tested pair counts as a candidate of its
    // primitive kind.
    int compound_narrow(Out<T>* o, int a, int b, V3<T> cB, T delta, int64_t* cnt) const {
        Shape<T> pa[MAX_CHILDREN], pb[MAX_CHILDREN];
        const int na = a >= 0 ? parts(a, mk<T>(0, 0, 0), pa) : 1;
        const int nb = parts(b, cB, pb);
        int first_hit = -1, idx = 0;
        double margin = 1e30;
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j, ++idx) {
                Out<T>& o2 = o[idx];
                if (!(a < 0 ? part_box_reaches_plane(pb[j], delta) : part_boxes_meet(pa[i], pb[j], delta))) continue;
                if (a < 0) {
                    narrow_plane(o2, T(0), pb[j], delta);
                    cnt[CNT_KIND0 + 9 + pb[j].type]++;
                } else {
                    narrow(o2, pa[i], pb[j], delta);
                    cnt[CNT_KIND0 + 3 * std::min(pa[i].type, pb[j].type) + std::max(pa[i].type, pb[j].type)]++;
                }
                reduce4(o2);
                if (o2.margin < margin) margin = o2.margin;
                if (o2.n > 0 && first_hit < 0) first_hit = idx;
            }
        o[0].decision = first_hit < 0 ? 63 : 64 + first_hit;
        o[0].margin = margin;
        return idx;
    }

    // S4 for one point set: a normal row per kept point (arms from the step-start centres) and the
    // manifold's friction patch at the points' centroid (tangent t1 along the pre-step sliding
    // velocity there, else the Duff et al. basis of the mean normal).
    void add_manifold(const Out<T>& o, int keep, int first, bool isplane, int a, int bb, V3<T> base, V3<T> offB,
                      int pair_index, int part, double& min_margin) {
        const Body<T>& A = E.bodies[a];
        int ia = isplane ? -1 : a, ib = isplane ? a : bb;
        T mu, e;
        if (isplane) { mu = (T(P.plane_friction) + A.mu) / T(2); e = std::max(T(P.plane_restitution), A.e); }
        else { mu = (A.mu + E.bodies[bb].mu) / T(2); e = std::max(A.e, E.bodies[bb].e); }
        V3<T> csum = mk<T>(0, 0, 0), nsum = mk<T>(0, 0, 0);
        for (int k = 0; k < keep; ++k) {
            CRow<T> r;
            r.a = ia; r.b = ib;
            V3<T> p = o.pt[k].p;  // relative to `base`
            r.n = o.pt[k].n;
            r.rA = ia >= 0 ? p : mk<T>(0, 0, 0);
            r.rB = p - offB;
            V3<T> vrel = vel_at(&E.bodies[ib], r.rB) - (ia >= 0 ? vel_at(&E.bodies[ia], r.rA) : mk<T>(0, 0, 0));
            r.vnpre = dot(vrel, r.n);
            r.mn = eff(ia, ib, r.rA, r.rB, r.n);
            r.s0 = o.pt[k].s;
            r.e = e;
            r.ln = 0;
            r.ln0 = 0;
            rows.push_back(r);
            csum = csum + p;
            nsum = nsum + r.n;
        }
        Manifold<T> M;
        M.a = ia; M.b = ib; M.first = first; M.count = keep; M.colour = 0; M.pair = pair_index; M.part = part;
        M.base = base; M.offB = offB;
        V3<T> c = (T(1) / T(keep)) * csum;
        M.nb = (T(1) / len(nsum)) * nsum;
        M.rA = ia >= 0 ? c : mk<T>(0, 0, 0);
        M.rB = c - offB;
        V3<T> vrel = vel_at(&E.bodies[ib], M.rB) - (ia >= 0 ? vel_at(&E.bodies[ia], M.rA) : mk<T>(0, 0, 0));
        V3<T> vt = vrel - dot(vrel, M.nb) * M.nb;
        T vtl = len(vt);
        if (std::fabs(double(vtl) - 1e-3) < min_margin) min_margin = std::fabs(double(vtl) - 1e-3);
        M.t1 = vtl >= T(1e-3) ? (T(1) / vtl) * vt : onb_t1(M.nb);
        M.t2 = cross(M.nb, M.t1);
        M.mt1 = eff(ia, ib, M.rA, M.rB, M.t1);
        M.mt2 = eff(ia, ib, M.rA, M.rB, M.t2);
        T kw = (ia >= 0 ? dot(M.nb, mul(bv[ia].Iw, M.nb)) : T(0)) + dot(M.nb, mul(bv[ib].Iw, M.nb));
        M.mtw = kw > T(0) ? T(1) / kw : T(0);
        T rsum = 0;
        for (int k = 0; k < keep; ++k) rsum = rsum + len(o.pt[k].p - c);
        M.rt = rsum / T(keep);
        M.mu = mu;
        M.lt1 = M.lt2 = M.ltw = 0;
        mans.push_back(M);
    }

    void prepare(double& min_margin, int64_t* cnt) {
        const int n = int(E.bodies.size());
        const T delta = T(P.contact_offset);
        bv.resize(n); x0.resize(n); q0.resize(n); dx.assign(n, mk<T>(0, 0, 0)); dq.assign(n, Q<T>{1, 0, 0, 0});
        for (int i = 0; i < n; ++i) {
            Body<T>& b = E.bodies[i];
            x0[i] = b.x; q0[i] = b.q;
            bv[i].invm = b.dyn() ? b.invm : T(0);
            bv[i].Iw = b.dyn() ? world_inv_inertia(b.q, b.invI) : M3<T>{};
            if (b.dyn()) cnt[CNT_DYN]++; else cnt[CNT_STATIC]++;
        }
        // S1: AABBs from the start-of-step pose; add, multiply, abs and compare only.
        std::vector<V3<T>> lo(n), hi(n);
        for (int i = 0; i < n; ++i) {
            const Body<T>& b = E.bodies[i];
            M3<T> R = rotm(b.q);
            V3<T> half;
            if (b.shape == COMPOUND) {
                // the largest extent over the parts: |R c_k| + the part's own half size
                const Compound<T>& C = (*E.comps)[b.comp];
                T hm[3] = {0, 0, 0};
                for (int k = 0; k < C.n; ++k) {
                    const V3<T> o = mul(R, C.c[k]);
                    const M3<T> Rk = rotm(qmul(b.q, C.q[k]));
                    for (int r = 0; r < 3; ++r) {
                        const T hv = std::fabs(get(o, r)) + part_half(C.shape[k], C.dims[k], Rk, r);
                        if (hv > hm[r]) hm[r] = hv;
                    }
                }
                for (int r = 0; r < 3; ++r) set(half, r, hm[r] + delta);
            } else
            for (int r = 0; r < 3; ++r) set(half, r, part_half(b.shape, b.dims, R, r) + delta);
            lo[i] = b.x - half;
            hi[i] = b.x + half;
        }
        // Joint filter: parent-child pairs never collide.
        std::vector<uint64_t> jmask(n, 0);
        for (const Joint<T>& j : E.joints)
            if (j.parent >= 0) { jmask[j.parent] |= uint64_t(1) << j.child; jmask[j.child] |= uint64_t(1) << j.parent; }

        // Capacities from the dynamic body count: points min(6 n_dyn + 8, 384), manifolds
        // min(3 n_dyn + 4, 192), unless the parameters set them.  Beyond them, the pairs that
        // come later in canonical order lose their points and the env is flagged (status 2).
        int n_dyn = 0;
        for (int i = 0; i < n; ++i) n_dyn += E.bodies[i].dyn() ? 1 : 0;
        const int cap = P.max_contacts_per_env > 0 ? P.max_contacts_per_env : std::min(6 * n_dyn + 8, 384);
        const int mcap = P.max_manifolds_per_env > 0 ? P.max_manifolds_per_env : std::min(3 * n_dyn + 4, 192);
        rows.clear(); mans.clear();
        // S2 + S3 in canonical order: for each a, partners b = a+1 .. n-1, then the plane.
        for (int a = 0; a < n; ++a) {
            for (int bb = a + 1; bb <= n; ++bb) {
                bool isplane = bb == n;
                cnt[CNT_PAIRS_TESTED]++;
                const Body<T>& A = E.bodies[a];
                if (isplane) {
                    if (!P.plane_enabled || !A.dyn()) continue;
                    if (!(lo[a].z <= T(P.plane_z))) continue;
                } else {
                    const Body<T>& B = E.bodies[bb];
                    if (!A.dyn() && !B.dyn()) continue;
                    if (jmask[a] >> bb & 1) continue;
                    if (!(lo[a].x <= hi[bb].x && lo[bb].x <= hi[a].x && lo[a].y <= hi[bb].y && lo[bb].y <= hi[a].y &&
                          lo[a].z <= hi[bb].z && lo[bb].z <= hi[a].z))
                        continue;
                }
                cnt[CNT_CAND]++;
                Out<T> outs[MAX_CHILDREN * MAX_CHILDREN];
                Out<T>& o = outs[0];
                int nout = 1;
                int kind;
                V3<T> base, offB;  // contact points come relative to `base`; B's centre is at offB
                if (isplane) {
                    kind = 9 + A.shape;  // 9 plane-sphere, 10 plane-capsule, 11 plane-box
                    // frame: origin at (x, y) of the body on the ground plane
                    base = mk(A.x.x, A.x.y, T(P.plane_z));
                    offB = mk(T(0), T(0), A.x.z - T(P.plane_z));
                    if (A.shape == COMPOUND) {
                        kind = 12;
                        nout = compound_narrow(outs, -1, a, offB, delta, cnt);
                    } else {
                        Shape<T> sb = shape_of(a);
                        sb.c = offB;
                        narrow_plane(o, T(0), sb, delta);
                    }
                } else {
                    // frame: origin at A's centre (translation-invariant contact geometry)
                    base = A.x;
                    offB = E.bodies[bb].x - A.x;
                    int sa = A.shape, sb = E.bodies[bb].shape;
                    if (sa == COMPOUND || sb == COMPOUND) {
                        kind = 12;
                        nout = compound_narrow(outs, a, bb, offB, delta, cnt);
                    } else {
                        int lo_s = std::min(sa, sb), hi_s = std::max(sa, sb);
                        kind = lo_s * 3 + hi_s;  // 0 ss,1 sc,2 sb,4 cc,5 cb,8 bb
                        Shape<T> sa2 = shape_of(a), sb2 = shape_of(bb);
                        sa2.c = mk<T>(0, 0, 0);
                        sb2.c = offB;
                        narrow(o, sa2, sb2, delta);
                    }
                }
                if (kind < 12) {
                    cnt[CNT_KIND0 + kind]++;
                    reduce4(o);
                }
                if (o.margin < min_margin) min_margin = o.margin;
                int pair_index = rec ? int(rec->pairs.size()) : 0;
                const int decision = o.decision;
                const double pmargin = o.margin;
                int kept = 0;
                for (int t = 0; t < nout; ++t) {
                    Out<T>& ot = outs[t];
                    if (ot.n == 0) continue;
                    int first = int(rows.size());
                    int keep = ot.n;
                    // overflow keeps the first points / manifolds in canonical order
                    if (first + keep > cap) { keep = cap - first; E.status |= ST_CONTACT_OVERFLOW; }
                    if (keep > 0 && int(mans.size()) >= mcap) { keep = 0; E.status |= ST_CONTACT_OVERFLOW; }
                    if (keep <= 0) continue;
                    kept += keep;
                    add_manifold(ot, keep, first, isplane, a, bb, base, offB, pair_index, t, min_margin);
                }
                if (rec) rec->pairs.push_back(PairRec{env_id, a, isplane ? PLANE_ID : bb, kept, decision, kind, pmargin,
                                                      0, 0, 0, 0, 0});
            }
        }
        if (P.warm_start) warm_from_cache();
        cnt[CNT_POINTS] += int64_t(rows.size());
        cnt[CNT_MANIFOLDS] += int64_t(mans.size());
        cnt[CNT_JOINTS] += int64_t(E.joints.size());
        // S5: greedy colouring over blocks = joints (index order) ++ manifolds (canonical order).
        std::vector<uint64_t> used(n, 0);
        order.clear();
        const int nj = int(E.joints.size());
        std::vector<int> colour(nj + mans.size(), 0);
        ncol = 0;
        bool overflow = false;
        for (int bidx = 0; bidx < int(colour.size()); ++bidx) {
            int a, b;
            if (bidx < nj) { a = E.joints[bidx].parent; b = E.joints[bidx].child; }
            else { a = mans[bidx - nj].a; b = mans[bidx - nj].b; }
            uint64_t u = 0;
            if (dyn(a)) u |= used[a];
            if (dyn(b)) u |= used[b];
            int c = 0;
            while (c < MAX_COLORS && (u >> c & 1)) ++c;
            if (c >= MAX_COLORS) { overflow = true; c = MAX_COLORS; }
            else {
                if (dyn(a)) used[a] |= uint64_t(1) << c;
                if (dyn(b)) used[b] |= uint64_t(1) << c;
            }
            colour[bidx] = c;
            if (c + 1 > ncol) ncol = c + 1;
        }
        if (overflow) E.status |= ST_COLOR_OVERFLOW;
        cnt[CNT_COLOURS] += ncol;
        for (int c = 0; c <= MAX_COLORS; ++c)
            for (int bidx = 0; bidx < int(colour.size()); ++bidx)
                if (colour[bidx] == c) order.push_back({c, bidx});
        for (int m = 0; m < int(mans.size()); ++m) mans[m].colour = colour[nj + m];
        if (rec)
            for (int bidx = 0; bidx < int(colour.size()); ++bidx)
                rec->blocks.push_back(BlockRec{env_id, bidx < nj ? 0 : 1, bidx < nj ? bidx : bidx - nj, colour[bidx]});
        js.assign(nj, JState<T>{{0, 0, 0}, {0, 0, 0}, 0, {0, 0}});
    }

    // ------------------------------------------------------------- joint block
    // Frames of a joint from the current poses: arms rA = R(qA) aA, rB = R(qB) aB, the axes b1,
    // b2, zA of the parent's joint frame (columns of R(qA QA)) and the anchors' separation
    // d = (xB + rB) - (xA + rA).  A prismatic joint's parent arm reaches the child anchor,
    // rA + d, so that its rows act at one point on both bodies.
    struct JFrame { int a, b; V3<T> rA, rB, zA, b1, b2, d; };
    JFrame jframe(const Joint<T>& j) const {
        JFrame f;
        f.a = j.parent; f.b = j.child;
        Q<T> qa = j.parent >= 0 ? E.bodies[j.parent].q : Q<T>{1, 0, 0, 0};
        const Body<T>& B = E.bodies[j.child];
        f.rA = rotate(qa, j.aA);
        f.rB = rotate(B.q, j.aB);
        M3<T> Ra = rotm(qmul(qa, j.QA));
        f.zA = col(Ra, 2); f.b1 = col(Ra, 0); f.b2 = col(Ra, 1);
        f.d = (pos_of(f.b) + f.rB) - (pos_of(f.a) + f.rA);
        if (j.type == PRISMATIC) f.rA = f.rA + f.d;
        return f;
    }
    V3<T> pos_of(int i) const { return i >= 0 ? E.bodies[i].x : mk<T>(0, 0, 0); }
    V3<T> lin_of(int i) const { return i >= 0 ? E.bodies[i].v : mk<T>(0, 0, 0); }
    V3<T> ang_of(int i) const { return i >= 0 ? E.bodies[i].w : mk<T>(0, 0, 0); }

    // Joint position: the twist of the child's joint frame relative to the parent's about zA,
    // 2 atan2(q_rel.z, q_rel.w) with q_rel.w >= 0 (revolute), or the anchors' separation along
    // the slide axis, zA . d (prismatic).
    T joint_pos(const Joint<T>& j, const JFrame& f) const {
        if (j.type == PRISMATIC) return dot(f.zA, f.d);
        Q<T> qa = j.parent >= 0 ? E.bodies[j.parent].q : Q<T>{1, 0, 0, 0};
        Q<T> rel = qmul(qconj(qmul(qa, j.QA)), qmul(E.bodies[j.child].q, j.QB));
        if (rel.w < T(0)) rel = Q<T>{-rel.w, -rel.x, -rel.y, -rel.z};
        return T(2) * atan2_pos(rel.z, rel.w);
    }
    // Drive error: joint position minus target; an angle is wrapped into (-pi, pi].
    T drive_error(const Joint<T>& j, const JFrame& f, T target) const {
        T c = joint_pos(j, f) - target;
        if (j.type == PRISMATIC) return c;
        // wrap into (-pi, pi] with the exact IEEE remainder (non-finite stays non-finite)
        const T pi = T(3.14159265358979323846);
        c = std::remainder(c, T(2) * pi);
        if (c <= -pi) c = c + T(2) * pi;
        return c;
    }
    // The joint's free axis zA as a row: inverse effective mass k of a unit impulse along it
    // (angular for a revolute joint, linear at the arms for a prismatic one), the relative
    // velocity along it, and the application of an impulse l along it (-l on A, +l on B).
    T axis_k(const Joint<T>& j, const JFrame& f) const {
        if (j.type == PRISMATIC) {
            T k = invm(f.a) + invm(f.b);
            if (f.a >= 0) { V3<T> c = cross(f.rA, f.zA); k = k + dot(c, mul(bv[f.a].Iw, c)); }
            V3<T> c = cross(f.rB, f.zA);
            return k + dot(c, mul(bv[f.b].Iw, c));
        }
        return dot(f.zA, mul(bv[f.b].Iw, f.zA)) + (f.a >= 0 ? dot(f.zA, mul(bv[f.a].Iw, f.zA)) : T(0));
    }
    T axis_vel(const Joint<T>& j, const JFrame& f) const {
        if (j.type == PRISMATIC)
            return dot(f.zA, (lin_of(f.b) + cross(ang_of(f.b), f.rB)) - (lin_of(f.a) + cross(ang_of(f.a), f.rA)));
        return dot(f.zA, ang_of(f.b) - ang_of(f.a));
    }
    void axis_apply(const Joint<T>& j, const JFrame& f, T l) {
        if (j.type == PRISMATIC) apply(f.a, f.b, f.rA, f.rB, l * f.zA);
        else apply_ang(f.a, f.b, l * f.zA);
    }

    void joint_warm(int ji) {
        const Joint<T>& j = E.joints[ji];
        JFrame f = jframe(j);
        JState<T>& s = js[ji];
        if (j.type == PRISMATIC) {
            apply(f.a, f.b, f.rA, f.rB, s.lp[0] * f.b1 + s.lp[1] * f.b2);
            apply_ang(f.a, f.b, mk(s.la[0], s.la[1], s.la[2]));
        } else {
            apply(f.a, f.b, f.rA, f.rB, mk(s.lp[0], s.lp[1], s.lp[2]));
            apply_ang(f.a, f.b, s.la[0] * f.b1 + s.la[1] * f.b2);
        }
        axis_apply(j, f, s.ld);
        if (j.limited) axis_apply(j, f, s.ll[0] - s.ll[1]);
    }

    // 3x3 solve lam = -K^-1 rhs by adjugate and determinant (no change when det = 0).
    static bool solve3(const M3<T>& K, V3<T> rhs, V3<T>& lam) {
        T c00 = K.m[1][1] * K.m[2][2] - K.m[1][2] * K.m[2][1];
        T c01 = K.m[0][2] * K.m[2][1] - K.m[0][1] * K.m[2][2];
        T c02 = K.m[0][1] * K.m[1][2] - K.m[0][2] * K.m[1][1];
        T c10 = K.m[1][2] * K.m[2][0] - K.m[1][0] * K.m[2][2];
        T c11 = K.m[0][0] * K.m[2][2] - K.m[0][2] * K.m[2][0];
        T c12 = K.m[0][2] * K.m[1][0] - K.m[0][0] * K.m[1][2];
        T c20 = K.m[1][0] * K.m[2][1] - K.m[1][1] * K.m[2][0];
        T c21 = K.m[0][1] * K.m[2][0] - K.m[0][0] * K.m[2][1];
        T c22 = K.m[0][0] * K.m[1][1] - K.m[0][1] * K.m[1][0];
        T det = K.m[0][0] * c00 + K.m[0][1] * c10 + K.m[0][2] * c20;
        if (det == T(0)) return false;
        T id = T(1) / det;
        lam = mk(-(c00 * rhs.x + c01 * rhs.y + c02 * rhs.z) * id, -(c10 * rhs.x + c11 * rhs.y + c12 * rhs.z) * id,
                 -(c20 * rhs.x + c21 * rhs.y + c22 * rhs.z) * id);
        return true;
    }
    // 2x2 symmetric solve (l1, l2) = -K^-1 (r1, r2) (no change when det = 0).
    static bool solve2(T k11, T k12, T k22, T r1, T r2, T& l1, T& l2) {
        T det = k11 * k22 - k12 * k12;
        if (det == T(0)) return false;
        T id = T(1) / det;
        l1 = -(k22 * r1 - k12 * r2) * id;
        l2 = -(-k12 * r1 + k11 * r2) * id;
        return true;
    }

    // Revolute: the anchors coincide (3x3 point block) and the joint axes stay aligned (2 angular
    // rows about b1, b2).
    void revolute_lock(const Joint<T>& j, const JFrame& f, JState<T>& st, T beta) {
        const int a = f.a, b = f.b;
        {
            M3<T> K{};
            T im = invm(a) + invm(b);
            for (int i = 0; i < 3; ++i) K.m[i][i] = im;
            auto add_arm = [&](V3<T> r, const M3<T>& I) {
                // subtract [r]x I [r]x
                M3<T> S{{{0, -r.z, r.y}, {r.z, 0, -r.x}, {-r.y, r.x, 0}}};
                M3<T> SI{}, SIS{};
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q)
                        SI.m[p][q] = S.m[p][0] * I.m[0][q] + S.m[p][1] * I.m[1][q] + S.m[p][2] * I.m[2][q];
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q)
                        SIS.m[p][q] = SI.m[p][0] * S.m[0][q] + SI.m[p][1] * S.m[1][q] + SI.m[p][2] * S.m[2][q];
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) K.m[p][q] = K.m[p][q] - SIS.m[p][q];
            };
            if (a >= 0) add_arm(f.rA, bv[a].Iw);
            add_arm(f.rB, bv[b].Iw);
            V3<T> Cd = (lin_of(b) + cross(ang_of(b), f.rB)) - (lin_of(a) + cross(ang_of(a), f.rA));
            V3<T> rhs = Cd + (beta / T(P.dt)) * f.d;
            V3<T> lam;
            if (solve3(K, rhs, lam)) {
                st.lp[0] = st.lp[0] + lam.x; st.lp[1] = st.lp[1] + lam.y; st.lp[2] = st.lp[2] + lam.z;
                apply(a, b, f.rA, f.rB, lam);
            }
        }
        {
            Q<T> qb = qmul(E.bodies[b].q, j.QB);
            V3<T> zB = col(rotm(qb), 2);
            V3<T> zc = cross(f.zA, zB);
            T C1 = dot(f.b1, zc), C2 = dot(f.b2, zc);
            V3<T> dw = ang_of(b) - ang_of(a);
            T Cd1 = dot(f.b1, dw), Cd2 = dot(f.b2, dw);
            M3<T> Isum{};
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) Isum.m[p][q] = (a >= 0 ? bv[a].Iw.m[p][q] : T(0)) + bv[b].Iw.m[p][q];
            T k11 = dot(f.b1, mul(Isum, f.b1)), k12 = dot(f.b1, mul(Isum, f.b2)), k22 = dot(f.b2, mul(Isum, f.b2));
            T r1 = Cd1 + (beta / T(P.dt)) * C1, r2 = Cd2 + (beta / T(P.dt)) * C2;
            T l1, l2;
            if (solve2(k11, k12, k22, r1, r2, l1, l2)) {
                st.la[0] = st.la[0] + l1; st.la[1] = st.la[1] + l2;
                apply_ang(a, b, l1 * f.b1 + l2 * f.b2);
            }
        }
    }

    // Prismatic: the rotation is locked (3 angular rows, error 2 vec(q_rel) in the parent's joint
    // frame, q_rel.w >= 0) and the child anchor stays on the slide line (2 rows along b1, b2 at
    // the arms rA + d and rB).
    void prismatic_lock(const Joint<T>& j, const JFrame& f, JState<T>& st, T beta) {
        const int a = f.a, b = f.b;
        {
            Q<T> qa = a >= 0 ? E.bodies[a].q : Q<T>{1, 0, 0, 0};
            Q<T> rel = qmul(qconj(qmul(qa, j.QA)), qmul(E.bodies[b].q, j.QB));
            if (rel.w < T(0)) rel = Q<T>{-rel.w, -rel.x, -rel.y, -rel.z};
            V3<T> e = (T(2) * rel.x) * f.b1 + (T(2) * rel.y) * f.b2 + (T(2) * rel.z) * f.zA;
            M3<T> K{};
            for (int p = 0; p < 3; ++p)
                for (int q = 0; q < 3; ++q) K.m[p][q] = (a >= 0 ? bv[a].Iw.m[p][q] : T(0)) + bv[b].Iw.m[p][q];
            V3<T> rhs = (ang_of(b) - ang_of(a)) + (beta / T(P.dt)) * e;
            V3<T> lam;
            if (solve3(K, rhs, lam)) {
                st.la[0] = st.la[0] + lam.x; st.la[1] = st.la[1] + lam.y; st.la[2] = st.la[2] + lam.z;
                apply_ang(a, b, lam);
            }
        }
        {
            const M3<T> Z{};
            const M3<T>& IA = a >= 0 ? bv[a].Iw : Z;
            const M3<T>& IB = bv[b].Iw;
            V3<T> cA1 = cross(f.rA, f.b1), cA2 = cross(f.rA, f.b2), cB1 = cross(f.rB, f.b1), cB2 = cross(f.rB, f.b2);
            T im = invm(a) + invm(b);
            T k11 = (im + dot(cA1, mul(IA, cA1))) + dot(cB1, mul(IB, cB1));
            T k12 = dot(cA1, mul(IA, cA2)) + dot(cB1, mul(IB, cB2));
            T k22 = (im + dot(cA2, mul(IA, cA2))) + dot(cB2, mul(IB, cB2));
            V3<T> vr = (lin_of(b) + cross(ang_of(b), f.rB)) - (lin_of(a) + cross(ang_of(a), f.rA));
            T r1 = dot(f.b1, vr) + (beta / T(P.dt)) * dot(f.b1, f.d);
            T r2 = dot(f.b2, vr) + (beta / T(P.dt)) * dot(f.b2, f.d);
            T l1, l2;
            if (solve2(k11, k12, k22, r1, r2, l1, l2)) {
                st.lp[0] = st.lp[0] + l1; st.lp[1] = st.lp[1] + l2;
                apply(a, b, f.rA, f.rB, l1 * f.b1 + l2 * f.b2);
            }
        }
    }

    void joint_solve(int ji, const T* targets, bool velocity_pass) {
        const Joint<T>& j = E.joints[ji];
        JFrame f = jframe(j);
        JState<T>& st = js[ji];
        const T beta = velocity_pass ? T(0) : T(P.joint_baumgarte);
        if (j.type == PRISMATIC) prismatic_lock(j, f, st, beta);
        else revolute_lock(j, f, st, beta);
        // PD drive as a soft row along the free axis
        if (j.kp != T(0) || j.kd != T(0)) {
            T k = axis_k(j, f);
            T den = j.kd + h * j.kp;
            T gamma = T(1) / (h * den);
            T beta_d = h * j.kp / den;
            T C = drive_error(j, f, targets[ji]);
            T Cd = axis_vel(j, f);
            T dl = -(Cd + beta_d * C / h + gamma * st.ld) / (k + gamma);
            st.ld = st.ld + dl;
            axis_apply(j, f, dl);
        }
        // Position limits: two one-sided rows along the free axis on the gaps s_lo = x - lower and
        // s_hi = upper - x; speculative (bias s / h) while the gap is open, Baumgarte at the
        // joint rate per step once it is closed, accumulated impulses >= 0.
        if (j.limited) {
            T k = axis_k(j, f);
            T m = k > T(0) ? T(1) / k : T(0);
            T x = joint_pos(j, f);
            for (int side = 0; side < 2; ++side) {
                T gap = side == 0 ? x - j.lower : j.upper - x;
                T bias = gap > T(0) ? gap / h : (velocity_pass ? T(0) : (T(P.joint_baumgarte) / T(P.dt)) * gap);
                T v = axis_vel(j, f);
                if (side == 1) v = -v;
                T nl = std::max(st.ll[side] - m * (v + bias), T(0));
                T dl = nl - st.ll[side];
                st.ll[side] = nl;
                axis_apply(j, f, side == 0 ? dl : -dl);
            }
        }
    }

    // ------------------------------------------------------------- manifold block
    // Displacement of the body-fixed point x0 + r since the step start: dx + R(dq) r - r, with
    // R(dq) r - r = 2 w (u x r) + 2 u x (u x r) for dq = (w, u) (no cancellation for small dq).
    V3<T> point_disp(int i, V3<T> r) const {
        const Q<T>& d = dq[i];
        V3<T> u = mk(d.x, d.y, d.z);
        V3<T> ur = cross(u, r);
        return dx[i] + (T(2) * d.w) * ur + T(2) * cross(u, ur);
    }
    T current_sep(const CRow<T>& r) const {
        V3<T> dA = r.a >= 0 ? point_disp(r.a, r.rA) : mk<T>(0, 0, 0);
        V3<T> dB = point_disp(r.b, r.rB);
        return r.s0 + dot(r.n, dB - dA);
    }
    V3<T> rel_vel(const CRow<T>& r) const {
        V3<T> vb = E.bodies[r.b].v + cross(E.bodies[r.b].w, r.rB);
        V3<T> va = r.a >= 0 ? E.bodies[r.a].v + cross(E.bodies[r.a].w, r.rA) : mk<T>(0, 0, 0);
        return vb - va;
    }
    V3<T> rel_vel_patch(const Manifold<T>& m) const {
        V3<T> vb = E.bodies[m.b].v + cross(E.bodies[m.b].w, m.rB);
        V3<T> va = m.a >= 0 ? E.bodies[m.a].v + cross(E.bodies[m.a].w, m.rA) : mk<T>(0, 0, 0);
        return vb - va;
    }
    void manifold_warm(const Manifold<T>& m) {
        for (int k = 0; k < m.count; ++k) {
            const CRow<T>& r = rows[m.first + k];
            apply(r.a, r.b, r.rA, r.rB, r.ln * r.n);
        }
        apply(m.a, m.b, m.rA, m.rB, m.lt1 * m.t1 + m.lt2 * m.t2);
        apply_ang(m.a, m.b, m.ltw * m.nb);
    }
    void manifold_solve(Manifold<T>& m, bool velocity_pass) {
        for (int k = 0; k < m.count; ++k) {
            CRow<T>& r = rows[m.first + k];
            T s = current_sep(r);
            T bias;
            if (s > T(0)) bias = s / h;
            else bias = velocity_pass ? T(0) : std::max(T(P.baumgarte) * s / h, -T(P.max_depen_vel));
            T vn = dot(rel_vel(r), r.n);
            T dl = -r.mn * (vn + bias);
            T nl = std::max(r.ln + dl, T(0));
            dl = nl - r.ln;
            r.ln = nl;
            apply(r.a, r.b, r.rA, r.rB, dl * r.n);
        }
        T lsum = 0;
        for (int k = 0; k < m.count; ++k) lsum = lsum + rows[m.first + k].ln;
        T lim = m.mu * lsum;
        {
            T vt = dot(rel_vel_patch(m), m.t1);
            T nl = m.lt1 - m.mt1 * vt;
            nl = std::min(std::max(nl, -lim), lim);
            T dl = nl - m.lt1;
            m.lt1 = nl;
            apply(m.a, m.b, m.rA, m.rB, dl * m.t1);
        }
        {
            T vt = dot(rel_vel_patch(m), m.t2);
            T nl = m.lt2 - m.mt2 * vt;
            nl = std::min(std::max(nl, -lim), lim);
            T dl = nl - m.lt2;
            m.lt2 = nl;
            apply(m.a, m.b, m.rA, m.rB, dl * m.t2);
        }
        {
            T limw = m.rt * lim;
            T wr = dot(m.nb, ang_of(m.b) - ang_of(m.a));
            T nl = m.ltw - m.mtw * wr;
            nl = std::min(std::max(nl, -limw), limw);
            T dl = nl - m.ltw;
            m.ltw = nl;
            apply_ang(m.a, m.b, dl * m.nb);
        }
    }

    void manifold_restitution(const Manifold<T>& m) {
        for (int k = 0; k < m.count; ++k) {
            CRow<T>& r = rows[m.first + k];
            if (!(r.vnpre < -T(P.bounce_threshold) && r.ln > T(0))) continue;
            T vn = dot(rel_vel(r), r.n);
            T dl = -r.mn * (vn + r.e * r.vnpre);
            T nl = std::max(r.ln + dl, T(0));
            dl = nl - r.ln;
            r.ln = nl;
            apply(r.a, r.b, r.rA, r.rB, dl * r.n);
        }
    }

    // Contact impulses of the step, per dynamic body (touch sensing): every substep's final
    // multipliers are that substep's impulses (the warm start re-applies the previous substep's,
    // the sweeps add to them), so the step's total is the sum over substeps 1 .. S-1 after their
    // sweeps plus the final multipliers after the velocity and restitution passes.  Each addition
    // takes the normal impulses of a body's points and the two tangent impulses of its friction
    // patches (added on the B side, subtracted on the A side; a body's manifolds in colour order,
    // the solver's order, points before the patch).  The twist impulse is a torque and is left
    // out; static bodies report no force.
    void accumulate_forces() {
        const int nj = int(E.joints.size());
        for (const auto& ob : order) {
            if (ob.second < nj) continue;
            const Manifold<T>& m = mans[ob.second - nj];
            const bool db = dyn(m.b), da = dyn(m.a);
            for (int k = 0; k < m.count; ++k) {
                const CRow<T>& r = rows[m.first + k];
                const V3<T> Pn = r.ln * r.n;
                if (db) E.force[m.b] = E.force[m.b] + Pn;
                if (da) E.force[m.a] = E.force[m.a] - Pn;
            }
            const V3<T> Pt = m.lt1 * m.t1 + m.lt2 * m.t2;
            if (db) E.force[m.b] = E.force[m.b] + Pt;
            if (da) E.force[m.a] = E.force[m.a] - Pt;
        }
    }

    void sweep(const T* targets, bool velocity_pass) {
        const int nj = int(E.joints.size());
        for (auto& ob : order) {
            int bidx = ob.second;
            if (bidx < nj) joint_solve(bidx, targets, velocity_pass);
            else manifold_solve(mans[bidx - nj], velocity_pass);
        }
    }

    // ------------------------------------------------------------- S0..S8 for one env
    void step(const T* targets, int64_t* cnt, double& min_margin) {
        const int n = int(E.bodies.size());
        std::vector<Body<T>> saved = E.bodies;
        prepare(min_margin, cnt);
        const bool tgs = P.solver == 0;
        const int S = tgs ? std::max(P.pos_iters, 1) : 1;
        const int K = tgs ? 1 : std::max(P.pos_iters, 1);
        h = T(P.dt) / T(S);
        const V3<T> g = mk(T(P.gravity[0]), T(P.gravity[1]), T(P.gravity[2]));
        const T ld = T(1) / (T(1) + h * T(P.lin_damping));
        const T ad = T(1) / (T(1) + h * T(P.ang_damping));
        const int nj = int(E.joints.size());
        E.force.assign(n, mk<T>(0, 0, 0));
        for (int s = 0; s < S; ++s) {
            for (int i = 0; i < n; ++i) {
                Body<T>& b = E.bodies[i];
                if (!b.dyn()) continue;
                b.v = ld * (b.v + h * g);
                b.w = ad * b.w;
            }
            // warm start: the previous substep's impulses; in the first substep, those taken from
            // the contact cache (joint impulses start from zero every step)
            if (s > 0 || P.warm_start)
                for (auto& ob : order) {
                    if (ob.second < nj) joint_warm(ob.second);
                    else manifold_warm(mans[ob.second - nj]);
                }
            for (int k = 0; k < K; ++k) {
                // joint_iters - 1 joint-only passes (colour order), then the full sweep
                for (int jx = 1; jx < P.joint_iters; ++jx)
                    for (auto& ob : order)
                        if (ob.second < nj) joint_solve(ob.second, targets, false);
                sweep(targets, false);
            }
            if (s + 1 < S) accumulate_forces();
            for (int i = 0; i < n; ++i) {
                Body<T>& b = E.bodies[i];
                if (!b.dyn()) continue;
                // symplectic Euler on the offsets from the step start: dx += h v and
                // dq <- normalise(dq + h/2 (0, w) dq); then x = x0 + dx, q = normalise(dq q0)
                dx[i] = dx[i] + h * b.v;
                Q<T> wq{T(0), b.w.x, b.w.y, b.w.z};
                Q<T> e = qmul(wq, dq[i]);
                T hh = T(0.5) * h;
                dq[i] = qnormalize(Q<T>{dq[i].w + hh * e.w, dq[i].x + hh * e.x, dq[i].y + hh * e.y, dq[i].z + hh * e.z});
                b.x = x0[i] + dx[i];
                b.q = qnormalize(qmul(dq[i], q0[i]));
            }
        }
        for (int k = 0; k < P.vel_iters; ++k) sweep(targets, true);
        for (auto& ob : order)
            if (ob.second >= nj) manifold_restitution(mans[ob.second - nj]);
        // S8: non-finite guard
        bool bad = false;
        for (int i = 0; i < n; ++i) {
            const Body<T>& b = E.bodies[i];
            T vals[13] = {b.x.x, b.x.y, b.x.z, b.q.w, b.q.x, b.q.y, b.q.z, b.v.x, b.v.y, b.v.z, b.w.x, b.w.y, b.w.z};
            for (T v : vals) if (!std::isfinite(double(v))) bad = true;
        }
        if (bad) { E.bodies = saved; E.status |= ST_NONFINITE; }
        if (P.warm_start) {
            if (bad) { E.cman.clear(); E.cpt.clear(); }
            else write_cache();
        }
        // net contact force averaged over the step: the step's contact impulses / dt (zero when
        // the step went non-finite)
        if (bad) E.force.assign(n, mk<T>(0, 0, 0));
        else {
            accumulate_forces();
            const T idt = T(1) / T(P.dt);
            for (V3<T>& f : E.force) f = idt * f;
        }
        if (rec) {
            for (const Manifold<T>& m : mans) {
                PairRec& pr = rec->pairs[m.pair];
                pr.lt1 = double(m.lt1); pr.lt2 = double(m.lt2); pr.ltw = double(m.ltw);
                pr.mu = double(m.mu); pr.rt = double(m.rt);
                for (int k = 0; k < m.count; ++k) {
                    const CRow<T>& r = rows[m.first + k];
                    V3<T> p = m.base + (r.a >= 0 ? r.rA : r.rB + m.offB);
                    rec->points.push_back(PointRec{env_id, m.pair, {double(p.x), double(p.y), double(p.z)},
                                                   {double(r.n.x), double(r.n.y), double(r.n.z)}, double(r.s0),
                                                   double(r.ln), double(r.ln0)});
                }
            }
        }
    }
};

// ----------------------------------------------------------------------------- batch handle
struct Handle {
    Params P;
    int prec;
    int n_envs;
    std::vector<int> body_off, joint_off;
    std::vector<Env<float>> ef;
    std::vector<Env<double>> ed;
    std::vector<float> targets;  // [total joints]
    std::vector<EnvRecord> recs;
    std::vector<Env<float>> ef0;   // initial state (resets)
    std::vector<Env<double>> ed0;
    std::vector<Compound<float>> cf;  // the compound table in each precision
    std::vector<Compound<double>> cd;
};

// Joint position (twist angle or slide) of joint j in env E's current state.
template <class T> static T joint_position(const Params& P, Env<T>& E, int j) {
    Stepper<T> st(P, E, nullptr, 0);
    typename Stepper<T>::JFrame f = st.jframe(E.joints[j]);
    return st.joint_pos(E.joints[j], f);
}

// Randomised reset of one env (the paper's reset randomisation: initial robot joint positions
// drawn around a reference configuration, objects' planar position and yaw drawn uniformly).
// From the initial state: every free dynamic body (the child of no joint) moves by
// xy_half * (2u - 1) in x and in y and turns about the world z axis through its centre by
// yaw_half * (2u - 1); every joint in index order takes the position q0 = q_init +
// joint_sigma * N (N from normal12) and poses its child from its parent (forward kinematics);
// all velocities are zero and the status is cleared; with targets_follow the joint's drive
// target becomes q0.  Draws: body i uses block (env, count, 1, i); joint j blocks (env, count, 0,
// 3j .. 3j + 2).  Returns -1 when a joint's parent is posed by a later joint.
struct ResetNoise { float joint_sigma, xy_half, yaw_half; int32_t targets_follow; };
template <class T> static int reset_env_random(const Params& P, Env<T>& E, Env<T>& init, int env_id,
                                               const ResetNoise& nz, uint64_t seed, uint32_t count, float* targets) {
    const int n = int(init.bodies.size()), nj = int(init.joints.size());
    std::vector<int> is_child(n, 0), posed(n, 0);
    for (const Joint<T>& j : init.joints) is_child[j.child] = 1;
    for (int i = 0; i < n; ++i) posed[i] = !is_child[i];
    for (const Joint<T>& j : init.joints) {
        if (j.parent >= 0 && !posed[j.parent]) return -1;
        posed[j.child] = 1;
    }
    std::vector<T> q_init(nj);
    for (int j = 0; j < nj; ++j) q_init[j] = joint_position(P, init, j);
    ResetStream rs{{uint32_t(seed & 0xFFFFFFFFu), uint32_t(seed >> 32)}, uint32_t(env_id), count};
    E.bodies = init.bodies;
    for (Body<T>& b : E.bodies) { b.v = mk<T>(0, 0, 0); b.w = mk<T>(0, 0, 0); }
    for (int i = 0; i < n; ++i) {
        Body<T>& b = E.bodies[i];
        if (!b.dyn() || is_child[i]) continue;
        uint32_t u[4];
        rs.draw(1, uint32_t(i), u);
        b.x.x = b.x.x + T(nz.xy_half) * (T(2) * unit24<T>(u[0]) - T(1));
        b.x.y = b.x.y + T(nz.xy_half) * (T(2) * unit24<T>(u[1]) - T(1));
        const T half = T(0.5) * (T(nz.yaw_half) * (T(2) * unit24<T>(u[2]) - T(1)));
        b.q = qnormalize(qmul(Q<T>{cos_series(half), T(0), T(0), sin_series(half)}, b.q));
    }
    for (int j = 0; j < nj; ++j) {
        const Joint<T>& J = E.joints[j];
        const T q0 = q_init[j] + T(nz.joint_sigma) * normal12<T>(rs, 0, uint32_t(3 * j));
        const Q<T> qp = J.parent >= 0 ? E.bodies[J.parent].q : Q<T>{1, 0, 0, 0};
        const V3<T> xp = J.parent >= 0 ? E.bodies[J.parent].x : mk<T>(0, 0, 0);
        const Q<T> qpf = qmul(qp, J.QA);
        const Q<T> rot = J.type == PRISMATIC ? Q<T>{1, 0, 0, 0}
                                             : Q<T>{cos_series(T(0.5) * q0), T(0), T(0), sin_series(T(0.5) * q0)};
        Body<T>& c = E.bodies[J.child];
        c.q = qnormalize(qmul(qmul(qpf, rot), qconj(J.QB)));
        V3<T> anchor = xp + rotate(qp, J.aA);
        if (J.type == PRISMATIC) anchor = anchor + q0 * col(rotm(qpf), 2);
        c.x = anchor - rotate(c.q, J.aB);
        if (nz.targets_follow && targets) targets[j] = float(q0);
    }
    E.status = 0;
    E.force.assign(n, mk<T>(0, 0, 0));
    E.cman.clear();
    E.cpt.clear();
    return 0;
}

template <class T> static void load_env(Env<T>& E, const BodyDesc* bd, int nb, const JointDesc* jd, int nj) {
    E.bodies.resize(nb);
    for (int i = 0; i < nb; ++i) {
        const BodyDesc& d = bd[i];
        Body<T>& b = E.bodies[i];
        b.shape = d.shape; b.flags = d.flags;
        for (int k = 0; k < 3; ++k) b.dims[k] = T(d.dims[k]);
        T m;
        V3<T> I;
        if (d.shape == COMPOUND) {
            b.comp = int(d.dims[0]);
            const Compound<T>& C = (*E.comps)[b.comp];
            m = d.mass > 0 ? T(d.mass) : T(d.density) * compound_volume(C);
            I = compound_inertia(C, m);
        } else {
            m = d.mass > 0 ? T(d.mass) : T(d.density) * shape_volume<T>(d.shape, b.dims);
            I = shape_inertia<T>(d.shape, b.dims, m);
        }
        if (b.flags & STATIC) { b.invm = 0; b.invI = mk<T>(0, 0, 0); }
        else { b.invm = T(1) / m; b.invI = mk(T(1) / I.x, T(1) / I.y, T(1) / I.z); }
        b.mu = T(d.friction); b.e = T(d.restitution);
        b.x = mk(T(d.pos[0]), T(d.pos[1]), T(d.pos[2]));
        b.q = Q<T>{T(d.quat[0]), T(d.quat[1]), T(d.quat[2]), T(d.quat[3])};
        b.v = mk(T(d.linvel[0]), T(d.linvel[1]), T(d.linvel[2]));
        b.w = mk(T(d.angvel[0]), T(d.angvel[1]), T(d.angvel[2]));
    }
    E.joints.resize(nj);
    for (int i = 0; i < nj; ++i) {
        const JointDesc& d = jd[i];
        Joint<T>& j = E.joints[i];
        j.parent = d.parent; j.child = d.child;
        j.aA = mk(T(d.frame_parent[0]), T(d.frame_parent[1]), T(d.frame_parent[2]));
        j.QA = Q<T>{T(d.frame_parent[3]), T(d.frame_parent[4]), T(d.frame_parent[5]), T(d.frame_parent[6])};
        j.aB = mk(T(d.frame_child[0]), T(d.frame_child[1]), T(d.frame_child[2]));
        j.QB = Q<T>{T(d.frame_child[3]), T(d.frame_child[4]), T(d.frame_child[5]), T(d.frame_child[6])};
        j.kp = T(d.kp); j.kd = T(d.kd); j.target = T(d.target);
        j.type = d.type;
        j.limited = d.limited != 0;
        j.lower = T(d.lower); j.upper = T(d.upper);
    }
    E.status = 0;
    E.force.assign(nb, mk<T>(0, 0, 0));
}

template <class T> static void run_env(Handle& H, std::vector<Env<T>>& envs, int e, int n_steps, bool record) {
    Env<T>& E = envs[e];
    EnvRecord& R = H.recs[e];
    std::vector<T> tg(E.joints.size());
    for (size_t j = 0; j < tg.size(); ++j) tg[j] = T(H.targets[H.joint_off[e] + j]);
    if (E.status & ST_NONFINITE) E.force.assign(E.bodies.size(), mk<T>(0, 0, 0));
    for (int s = 0; s < n_steps; ++s) {
        if (E.status & ST_NONFINITE) break;
        bool last = s == n_steps - 1;
        if (last && record) { R.pairs.clear(); R.points.clear(); R.blocks.clear(); }
        std::fill(R.cnt, R.cnt + N_CNT, 0);
        R.min_margin = 1e30;
        Stepper<T> st(H.P, E, (last && record) ? &R : nullptr, e);
        st.step(tg.data(), R.cnt, R.min_margin);
    }
}

template <class T> static void run_all(Handle& H, std::vector<Env<T>>& envs, int n_steps, int n_threads, bool record) {
    const int E = H.n_envs;
    if (n_threads <= 1) {
        for (int e = 0; e < E; ++e) run_env(H, envs, e, n_steps, record);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t)
        th.emplace_back([&, t]() {
            for (int e = t; e < E; e += n_threads) run_env(H, envs, e, n_steps, record);
        });
    for (auto& x : th) x.join();
}

// State in SoA over all bodies: pos[3][B], quat[4][B], v[3][B], w[3][B] (double), status[E].
template <class T> static void get_state_t(Handle* H, std::vector<Env<T>>& envs, double* pos, double* quat, double* v,
                                           double* w, int32_t* status) {
    const int B = H->body_off[H->n_envs];
    for (int e = 0; e < H->n_envs; ++e) {
        if (status) status[e] = envs[e].status;
        for (size_t i = 0; i < envs[e].bodies.size(); ++i) {
            const Body<T>& b = envs[e].bodies[i];
            int g = H->body_off[e] + int(i);
            pos[g] = double(b.x.x); pos[B + g] = double(b.x.y); pos[2 * B + g] = double(b.x.z);
            quat[g] = double(b.q.w); quat[B + g] = double(b.q.x); quat[2 * B + g] = double(b.q.y); quat[3 * B + g] = double(b.q.z);
            v[g] = double(b.v.x); v[B + g] = double(b.v.y); v[2 * B + g] = double(b.v.z);
            w[g] = double(b.w.x); w[B + g] = double(b.w.y); w[2 * B + g] = double(b.w.z);
        }
    }
}
template <class T> static void set_state_t(Handle* H, std::vector<Env<T>>& envs, const double* pos, const double* quat,
                                           const double* v, const double* w) {
    const int B = H->body_off[H->n_envs];
    for (int e = 0; e < H->n_envs; ++e) {
        envs[e].status = 0;
        envs[e].cman.clear();
        envs[e].cpt.clear();
        for (size_t i = 0; i < envs[e].bodies.size(); ++i) {
            Body<T>& b = envs[e].bodies[i];
            int g = H->body_off[e] + int(i);
            b.x = mk(T(pos[g]), T(pos[B + g]), T(pos[2 * B + g]));
            b.q = Q<T>{T(quat[g]), T(quat[B + g]), T(quat[2 * B + g]), T(quat[3 * B + g])};
            b.v = mk(T(v[g]), T(v[B + g]), T(v[2 * B + g]));
            b.w = mk(T(w[g]), T(w[B + g]), T(w[2 * B + g]));
        }
    }
}

template <class T> static void load_compounds(std::vector<Compound<T>>& out, const CompoundDesc* cd, int n) {
    out.resize(n);
    for (int i = 0; i < n; ++i) {
        Compound<T>& C = out[i];
        C.n = cd[i].n_children;
        for (int k = 0; k < C.n; ++k) {
            C.shape[k] = cd[i].shape[k];
            for (int r = 0; r < 3; ++r) C.dims[k][r] = T(cd[i].dims[k][r]);
            const float* ps = cd[i].pose[k];
            C.c[k] = mk(T(ps[0]), T(ps[1]), T(ps[2]));
            C.q[k] = Q<T>{T(ps[3]), T(ps[4]), T(ps[5]), T(ps[6])};
        }
    }
}

}  // namespace orc

using namespace orc;

extern "C" {

void* or_create(const Params* p, int n_envs, const int32_t* body_off, const BodyDesc* bodies,
                const int32_t* joint_off, const JointDesc* joints, int precision, int n_compounds,
                const CompoundDesc* compounds) {
    Handle* H = new Handle();
    H->P = *p;
    H->prec = precision;
    H->n_envs = n_envs;
    load_compounds(H->cf, compounds, n_compounds);
    load_compounds(H->cd, compounds, n_compounds);
    H->body_off.assign(body_off, body_off + n_envs + 1);
    H->joint_off.assign(joint_off, joint_off + n_envs + 1);
    if (precision == 64) H->ed.resize(n_envs); else H->ef.resize(n_envs);
    H->recs.resize(n_envs);
    for (int e = 0; e < n_envs; ++e) {
        int b0 = body_off[e], nb = body_off[e + 1] - b0, j0 = joint_off[e], nj = joint_off[e + 1] - j0;
        if (precision == 64) { H->ed[e].comps = &H->cd; load_env(H->ed[e], bodies + b0, nb, joints + j0, nj); }
        else { H->ef[e].comps = &H->cf; load_env(H->ef[e], bodies + b0, nb, joints + j0, nj); }
    }
    int nj = joint_off[n_envs];
    H->targets.resize(nj);
    for (int j = 0; j < nj; ++j) H->targets[j] = joints[j].target;
    H->ef0 = H->ef;
    H->ed0 = H->ed;
    return H;
}

void or_destroy(void* h) { delete static_cast<Handle*>(h); }

void or_set_targets(void* h, const float* t) {
    Handle* H = static_cast<Handle*>(h);
    std::copy(t, t + H->targets.size(), H->targets.begin());
}

void or_step(void* h, int n_steps, int n_threads, int record) {
    Handle* H = static_cast<Handle*>(h);
    if (H->prec == 64) run_all(*H, H->ed, n_steps, n_threads, record != 0);
    else run_all(*H, H->ef, n_steps, n_threads, record != 0);
}

void or_get_state(void* h, double* pos, double* quat, double* v, double* w, int32_t* status) {
    Handle* H = static_cast<Handle*>(h);
    if (H->prec == 64) get_state_t(H, H->ed, pos, quat, v, w, status);
    else get_state_t(H, H->ef, pos, quat, v, w, status);
}
void or_set_state(void* h, const double* pos, const double* quat, const double* v, const double* w) {
    Handle* H = static_cast<Handle*>(h);
    if (H->prec == 64) set_state_t(H, H->ed, pos, quat, v, w);
    else set_state_t(H, H->ef, pos, quat, v, w);
}

// Test record of the last recorded step.
void or_record_sizes(void* h, int64_t* n_pairs, int64_t* n_points, int64_t* n_blocks) {
    Handle* H = static_cast<Handle*>(h);
    int64_t a = 0, b = 0, c = 0;
    for (auto& r : H->recs) { a += int64_t(r.pairs.size()); b += int64_t(r.points.size()); c += int64_t(r.blocks.size()); }
    *n_pairs = a; *n_points = b; *n_blocks = c;
}
// pairs: int32 [n][6] = env, a, b, npts, decision, kind; double [n][6] = decision margin and the
// friction patch's lambda_t1, lambda_t2, lambda_twist, mu, torsional radius
void or_record_pairs(void* h, int32_t* out, double* margin) {
    Handle* H = static_cast<Handle*>(h);
    int64_t k = 0;
    for (auto& r : H->recs)
        for (auto& p : r.pairs) {
            int32_t* o = out + 6 * k;
            o[0] = p.env; o[1] = p.a; o[2] = p.b; o[3] = p.npts; o[4] = p.decision; o[5] = p.kind;
            double* m = margin + 6 * k;
            m[0] = p.margin; m[1] = p.lt1; m[2] = p.lt2; m[3] = p.ltw; m[4] = p.mu; m[5] = p.rt;
            ++k;
        }
}
// points: int32 [n][2] = env, pair index (within the env's pair list); double [n][8] =
// p(3), n(3), s0, lambda_n
void or_record_points(void* h, int32_t* ids, double* out) {
    Handle* H = static_cast<Handle*>(h);
    int64_t k = 0;
    for (auto& r : H->recs)
        for (auto& p : r.points) {
            ids[2 * k] = p.env; ids[2 * k + 1] = p.pair;
            double* o = out + 9 * k;
            for (int i = 0; i < 3; ++i) { o[i] = p.p[i]; o[3 + i] = p.n[i]; }
            o[6] = p.s; o[7] = p.ln; o[8] = p.ln0;
            ++k;
        }
}
// blocks: int32 [n][4] = env, kind (0 joint, 1 manifold), index, colour
void or_record_blocks(void* h, int32_t* out) {
    Handle* H = static_cast<Handle*>(h);
    int64_t k = 0;
    for (auto& r : H->recs)
        for (auto& b : r.blocks) {
            int32_t* o = out + 4 * k;
            o[0] = b.env; o[1] = b.kind; o[2] = b.index; o[3] = b.colour;
            ++k;
        }
}
// Per-env work counters of the last step: int64 [E][N_CNT]; per-env minimum decision margin [E].
int or_n_counters() { return N_CNT; }
void or_env_counters(void* h, int64_t* out, double* min_margin) {
    Handle* H = static_cast<Handle*>(h);
    for (int e = 0; e < H->n_envs; ++e) {
        for (int c = 0; c < N_CNT; ++c) out[int64_t(e) * N_CNT + c] = H->recs[e].cnt[c];
        min_margin[e] = H->recs[e].min_margin;
    }
}

// Randomised reset of the listed envs (noise = joint_sigma, xy_half, yaw_half); returns 0, or
// -1 when an env's joints are not ordered parents first (nothing is changed then).
int or_reset_random(void* h, const int32_t* env_ids, int n_ids, const float* noise, int targets_follow, uint64_t seed,
                    uint32_t count) {
    Handle* H = static_cast<Handle*>(h);
    ResetNoise nz{noise[0], noise[1], noise[2], targets_follow};
    for (int k = 0; k < n_ids; ++k) {
        const int e = env_ids[k];
        if (e < 0 || e >= H->n_envs) continue;
        float* tg = H->targets.data() + H->joint_off[e];
        int r = H->prec == 64 ? reset_env_random(H->P, H->ed[e], H->ed0[e], e, nz, seed, count, tg)
                              : reset_env_random(H->P, H->ef[e], H->ef0[e], e, nz, seed, count, tg);
        if (r != 0) return r;
    }
    return 0;
}

// Target delta joint position controller: target += clip(a, -1, 1) (high - low) / 2 per joint
// (low / high per joint, or the scalars when the arrays are null), in float32 like the targets.
void or_apply_actions(void* h, const float* actions, const float* low, const float* high, float lo, float hi) {
    Handle* H = static_cast<Handle*>(h);
    for (size_t j = 0; j < H->targets.size(); ++j) {
        const float a = actions[j];
        const float c = a < -1.0f ? -1.0f : (a > 1.0f ? 1.0f : a);
        const float l = low ? low[j] : lo, u = high ? high[j] : hi;
        H->targets[j] = H->targets[j] + c * (0.5f * (u - l));
    }
}
void or_get_targets(void* h, float* out) {
    Handle* H = static_cast<Handle*>(h);
    std::copy(H->targets.begin(), H->targets.end(), out);
}

// Current joint positions [J] and net contact forces of the last step [3][B] (double).
void or_joint_positions(void* h, double* out) {
    Handle* H = static_cast<Handle*>(h);
    for (int e = 0; e < H->n_envs; ++e)
        for (int j = H->joint_off[e]; j < H->joint_off[e + 1]; ++j)
            out[j] = H->prec == 64 ? joint_position(H->P, H->ed[e], j - H->joint_off[e])
                                   : double(joint_position(H->P, H->ef[e], j - H->joint_off[e]));
}
void or_contact_forces(void* h, double* out) {
    Handle* H = static_cast<Handle*>(h);
    const int B = H->body_off[H->n_envs];
    for (int e = 0; e < H->n_envs; ++e) {
        const int nb = H->body_off[e + 1] - H->body_off[e];
        for (int i = 0; i < nb; ++i) {
            const int g = H->body_off[e] + i;
            double f[3] = {0, 0, 0};
            if (H->prec == 64) { const auto& v = H->ed[e].force[i]; f[0] = v.x; f[1] = v.y; f[2] = v.z; }
            else { const auto& v = H->ef[e].force[i]; f[0] = v.x; f[1] = v.y; f[2] = v.z; }
            out[g] = f[0]; out[B + g] = f[1]; out[2 * B + g] = f[2];
        }
    }
}

// The random-draw building blocks, exposed for the pins.
void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }
double or_sin_series(double x, int precision) { return precision == 64 ? sin_series<double>(x) : double(sin_series<float>(float(x))); }
double or_cos_series(double x, int precision) { return precision == 64 ? cos_series<double>(x) : double(cos_series<float>(float(x))); }
double or_normal12(uint64_t seed, uint32_t env, uint32_t count, uint32_t purpose, uint32_t first_block, int precision) {
    ResetStream rs{{uint32_t(seed & 0xFFFFFFFFu), uint32_t(seed >> 32)}, env, count};
    return precision == 64 ? normal12<double>(rs, purpose, first_block) : double(normal12<float>(rs, purpose, first_block));
}

// The drive's arctangent, exposed for the pins (float64 and float32).
double or_atan2_pos64(double y, double x) { return atan2_pos<double>(y, x); }
float or_atan2_pos32(float y, float x) { return atan2_pos<float>(y, x); }

// Mass properties exposed for the pins: volume and principal inertia for a given mass.
void or_mass_props(int shape, const double* dims, double mass, double* volume, double* inertia) {
    *volume = shape_volume<double>(shape, dims);
    V3<double> I = shape_inertia<double>(shape, dims, mass);
    inertia[0] = I.x; inertia[1] = I.y; inertia[2] = I.z;
}

// Volume and principal moments of a compound (mass `mass`) in float64, as the step uses them.
void or_compound_props(const CompoundDesc* cd, double mass, double* volume, double* inertia) {
    std::vector<Compound<double>> c;
    load_compounds(c, cd, 1);
    *volume = compound_volume(c[0]);
    V3<double> I = compound_inertia(c[0], mass);
    inertia[0] = I.x; inertia[1] = I.y; inertia[2] = I.z;
}

// Narrowphase for one pair of free-standing shapes (A = shape a, B = shape b, n from A to B);
// shape -1 means the ground plane at z = 0 (always A).  pose = (px, py, pz, qw, qx, qy, qz).
// Returns the number of points written as double [k][7] = p, n, s.  *decision receives the
// branch code.
int or_narrow(int shape_a, const double* dims_a, const double* pose_a, int shape_b, const double* dims_b,
              const double* pose_b, double delta, double* out, int32_t* decision) {
    auto mkshape = [](int s, const double* d, const double* p) {
        Shape<double> r;
        r.type = s;
        r.c = mk(p[0], p[1], p[2]);
        r.R = rotm(Q<double>{p[3], p[4], p[5], p[6]});
        r.d[0] = d[0]; r.d[1] = d[1]; r.d[2] = d[2];
        return r;
    };
    Out<double> o;
    Shape<double> B = mkshape(shape_b, dims_b, pose_b);
    if (shape_a < 0) narrow_plane(o, 0.0, B, delta);
    else narrow(o, mkshape(shape_a, dims_a, pose_a), B, delta);
    reduce4(o);
    for (int k = 0; k < o.n; ++k) {
        double* r = out + 7 * k;
        r[0] = o.pt[k].p.x; r[1] = o.pt[k].p.y; r[2] = o.pt[k].p.z;
        r[3] = o.pt[k].n.x; r[4] = o.pt[k].n.y; r[5] = o.pt[k].n.z;
        r[6] = o.pt[k].s;
    }
    *decision = o.decision;
    return o.n;
}

// Manifold reduction of n <= 16 points (double [n][4] = p, s; normal +z) for the pins: writes
// the indices picked in selection order (deepest, farthest, largest triangle, largest added
// area) to picked[4] and returns the number of points kept (picked is untouched when n <= 4).
int or_reduce4(const double* pts, int n, int32_t* picked) {
    Out<double> o;
    o.n = n < 16 ? n : 16;
    for (int k = 0; k < o.n; ++k) o.pt[k] = Pt<double>{mk(pts[4 * k], pts[4 * k + 1], pts[4 * k + 2]), mk(0.0, 0.0, 1.0),
                                                       pts[4 * k + 3]};
    int pk[4] = {-1, -1, -1, -1};
    reduce4(o, pk);
    for (int k = 0; k < 4; ++k) picked[k] = pk[k];
    return o.n;
}

// Separating-axis values of two boxes (15 axes: A faces, B faces, A_i x B_j), float64, for the
// pins: sep[k] = gap along axis k (negative = overlap), valid[k] = 0 for a degenerate cross.
void or_box_box_sat(const double* dims_a, const double* pose_a, const double* dims_b, const double* pose_b,
                    double* sep, int32_t* valid) {
    auto mkbox = [](const double* d, const double* p) {
        Shape<double> r;
        r.type = BOX;
        r.c = mk(p[0], p[1], p[2]);
        r.R = rotm(Q<double>{p[3], p[4], p[5], p[6]});
        r.d[0] = d[0]; r.d[1] = d[1]; r.d[2] = d[2];
        return r;
    };
    Shape<double> A = mkbox(dims_a, pose_a), B = mkbox(dims_b, pose_b);
    V3<double> d = B.c - A.c;
    for (int k = 0; k < 15; ++k) {
        V3<double> L;
        if (k < 3) L = col(A.R, k);
        else if (k < 6) L = col(B.R, k - 3);
        else {
            L = cross(col(A.R, (k - 6) / 3), col(B.R, (k - 6) % 3));
            double l = len(L);
            if (l < 1e-6) { valid[k] = 0; sep[k] = -1e30; continue; }
            L = (1.0 / l) * L;
        }
        valid[k] = 1;
        sep[k] = std::fabs(dot(d, L)) - box_extent(A, L) - box_extent(B, L);
    }
}

}  // extern "C"


// ms_host.cpp — host runtime of libms: validation, workspace layout, env-tile planning,
// launches and the C ABI declared in include/ms.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <memory>
#include <thread>
#include <vector>

#include "ms.h"
#include "ms_dev.h"

static_assert(sizeof(ms_body_desc) == 88 && sizeof(ms_joint_desc) == 92 && sizeof(ms_sim_params) == 96,
              "descriptor layouts are part of the ABI");

using namespace msdev;

extern "C" __global__ void ms_step_kernel(const BatchDev* batches, const Tile* tiles, int n_tiles, const TileEnv* tenv,
                                          int n_steps);
extern "C" __global__ void ms_step_kernel_w2(const BatchDev* batches, const Tile* tiles, int n_tiles,
                                             const TileEnv* tenv, int n_steps);
extern "C" __global__ void ms_step_kernel_one(const BatchDev* batches, const Tile* tiles, int n_tiles,
                                              const TileEnv* tenv, int n_steps);
extern "C" __global__ void ms_step_kernel_one_w2(const BatchDev* batches, const Tile* tiles, int n_tiles,
                                                 const TileEnv* tenv, int n_steps);
extern "C" __global__ void ms_reset_kernel(BatchDev bd, const int* env_ids, int n_ids, const float* spos,
                                           const float* squat, const float* svel, const float* sang);

namespace {

thread_local std::string g_err;

ms_status fail(ms_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ms_status fail(ms_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_OK(call)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return fail(MS_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

constexpr int MAX_CLASSES = 4;  // one stream per class; the default four hardware queues
constexpr int BIN_BUDGET = 20480;   // default bin LDS budget in words: half a CU's 160 KiB, two bins per CU

// Per-env sizes used by the planner.
struct EnvInfo {
    int n, nj, n_dyn, cap, mcap, words, lanes;
    float cost;   // estimated work of a step (launch order only)
};

// Lanes per env: enough lanes for the env's parallel work, then widened until 64 / G envs of
// this size fit the tile LDS budget.
int pick_lanes(const EnvInfo& e, int forced, int tile_budget_words) {
    if (forced > 0) return forced;
    int G;
    if (e.n <= 2 && e.nj == 0) G = 8;
    else if (e.n <= 10) G = 16;
    else if (e.n <= 14) G = 32;
    else G = 64;
    while (G < 64 && (WAVE / G) * e.words > tile_budget_words) G *= 2;
    return G;
}

// Tiles of one LDS class run in one launch whose dynamic LDS is the class maximum.
// A class is launched on its own stream as up to two kernels in sequence: its one-env, 64-lane
// tiles (the first n_one) with a scalar-env build, the other tiles with a general build.
struct LdsClass {
    int first_tile, n_tiles, lds_words;
    int variant;  // of the one-env part: 2 ms_step_kernel_one, 3 ms_step_kernel_one_w2
    int lanes;    // lanes per env of the class's first tile
    int n_one;    // leading one-env tiles
    int variant_gen;  // of the rest: 0 ms_step_kernel, 1 ms_step_kernel_w2 (two waves per SIMD)
};

typedef void (*StepKernel)(const BatchDev*, const Tile*, int, const TileEnv*, int);
// Kernel of a variant for a feature level: 0 the plain build, 1 the twin that carries the
// optional phases (contact forces, contact cache), 3 the one that also handles compound bodies.
inline StepKernel kernel_of(int variant, int feat) {
    static const StepKernel k[3][4] = {
        {ms_step_kernel, ms_step_kernel_w2, ms_step_kernel_one, ms_step_kernel_one_w2},
        {ms_step_kernel_opt, ms_step_kernel_w2_opt, ms_step_kernel_one_opt, ms_step_kernel_one_w2_opt},
        {ms_step_kernel_comp, ms_step_kernel_w2_comp, ms_step_kernel_one_comp, ms_step_kernel_one_w2_comp}};
    const int f = feat >= 2 ? 2 : (feat > 0 ? 1 : 0);
    return k[f][variant >= 0 && variant < 4 ? variant : 0];
}
typedef void (*BinsKernel)(const BatchDev*, const Tile*, const Bin*, int, const TileEnv*, int);
inline BinsKernel bins_kernel(int feat) {
    return feat >= 2 ? ms_step_kernel_bins_comp : (feat > 0 ? ms_step_kernel_bins_opt : ms_step_kernel_bins);
}
inline bool one_env_tile(const Tile& t) { return t.lanes == WAVE && t.count == 1; }

// Cut tiles sorted by LDS need (largest first) into launch classes — a new class when a tile
// needs less than 2/3 of the class maximum, at most MAX_CLASSES.  Default kernels: two waves per SIMD for the one-env part; for
// the rest, two waves per SIMD in a class that starts with 64-lane tiles (large envs), else the
// unconstrained build.
// A vector over caller storage of fixed capacity (the planner's containers in the entry point
// that allocates nothing); push_back past the capacity is a programming error, checked by the
// callers' size bounds.
template <class T>
struct FixedVec {
    T* d;
    size_t cap, n = 0;
    FixedVec(T* data, size_t capacity) : d(data), cap(capacity) {}
    void clear() { n = 0; }
    bool empty() const { return n == 0; }
    size_t size() const { return n; }
    void push_back(const T& v) { d[n++] = v; }
    T& back() { return d[n - 1]; }
    T& operator[](size_t i) { return d[i]; }
    const T& operator[](size_t i) const { return d[i]; }
    T* begin() { return d; }
    T* end() { return d + n; }
};

template <class TileRef, class ClassVec>
void cut_classes(int n, TileRef tile_ref, bool split_ok, ClassVec& cls) {
    cls.clear();
    for (int t = 0; t < n; ++t) {
        const Tile& tl = tile_ref(t);
        bool split = !cls.empty() && split_ok && int(cls.size()) < MAX_CLASSES &&
                     3 * tl.lds_words < 2 * cls.back().lds_words;
        if (cls.empty() || split) cls.push_back(LdsClass{t, 0, tl.lds_words, 3, tl.lanes, 0, tl.lanes == WAVE ? 1 : 0});
        cls.back().n_tiles++;
        cls.back().lds_words = std::max(cls.back().lds_words, tl.lds_words);
    }
    // a class made only of one-env tiles runs the scalar-env build; a mixed class runs the
    // general build on all its tiles (two launches in sequence on one stream cost more tail
    // than the scalar-env build saves)
    for (LdsClass& c : cls) {
        bool all_one = true;
        for (int t = c.first_tile; t < c.first_tile + c.n_tiles; ++t) all_one = all_one && one_env_tile(tile_ref(t));
        c.n_one = all_one ? c.n_tiles : 0;
    }
}

// Launch one class on stream s: the one-env part, then the general part.
ms_status launch_class(const LdsClass& c, const BatchDev* dbd, const Tile* tiles, const TileEnv* tenv, int n_steps,
                       int grid_cap, hipStream_t s, int opt) {
    const size_t lds = size_t(c.lds_words) * 4;
    const int parts[2][3] = {{c.first_tile, c.n_one, c.variant},
                             {c.first_tile + c.n_one, c.n_tiles - c.n_one, c.variant_gen}};
    for (const auto& pt : parts) {
        if (pt[1] <= 0) continue;
        const int grid = grid_cap > 0 ? std::max(1, std::min(pt[1], grid_cap)) : pt[1];
        hipLaunchKernelGGL(kernel_of(pt[2], opt), dim3(grid), dim3(WAVE), lds, s, dbd, tiles + pt[0], pt[1], tenv, n_steps);
        HIP_OK(hipGetLastError());
    }
    return MS_OK;
}

struct Plan {
    std::vector<EnvInfo> info;
    std::vector<Tile> tiles;  // ordered by LDS class, largest first
    std::vector<TileEnv> tenv;
    std::vector<LdsClass> classes;
    int max_tile_words = 0;
    // single-launch form (batches whose tiles fall into several LDS classes): bins of up to
    // BIN_WAVES tiles packed first-fit by decreasing size into one workgroup's LDS
    std::vector<Bin> bins;
    int bin_words = 0;
    int bin_tiles = BIN_WAVES;     // bin shape: at most this many tiles (wavefronts) per bin
    int bin_budget = BIN_BUDGET;   // and this many LDS words, unless one tile needs more
    int launch_mode = 0;   // 0: bins when several LDS classes, 1: always class launches
    // debug offsets
    std::vector<int> dbg_pair_off, dbg_pt_off, dbg_man_off;
};

// Workspace sections (byte offsets from the workspace base).
struct WsLayout {
    size_t pos, quat, vel, angvel, ipos, iquat, ivel, iang, save, status, bpar, body_off, joint_off, jrec, targets, tiles,
        bins, tenv, bd, stats, forces, bad_ids, phase_clock, comp, cache_hdr, cache_man, cache_man_off, cache_pt, cache_pt_off, cache_save,
        cache_bytes, dbg_pairs, dbg_pair_off, dbg_pts, dbg_pt_off, dbg_man, dbg_man_off, dbg_counts, total;
};

// Volume and principal moments of a primitive about its centre, float32, in the step model's
// order of operations (uniform density).
float prim_volume(int shape, const float* d) {
    const float fpi = 3.14159265358979323846f;
    if (shape == MS_SPHERE) return 4.0f / 3.0f * fpi * d[0] * d[0] * d[0];
    if (shape == MS_CAPSULE) { float L = 2.0f * d[1]; return fpi * d[0] * d[0] * L + 4.0f / 3.0f * fpi * d[0] * d[0] * d[0]; }
    return 8.0f * d[0] * d[1] * d[2];
}
void prim_inertia(int shape, const float* d, float m, float I[3]) {
    const float f0 = d[0], f1 = d[1], f2 = d[2];
    if (shape == MS_SPHERE) { float i = 2.0f / 5.0f * m * f0 * f0; I[0] = I[1] = I[2] = i; }
    else if (shape == MS_BOX) {
        float a = 2.0f * f0, bb = 2.0f * f1, c = 2.0f * f2;
        I[0] = m / 12.0f * (bb * bb + c * c); I[1] = m / 12.0f * (a * a + c * c); I[2] = m / 12.0f * (a * a + bb * bb);
    } else {
        const float fpi = 3.14159265358979323846f;
        float r = f0, L = 2.0f * f1;
        float vc = fpi * r * r * L, vs = 4.0f / 3.0f * fpi * r * r * r;
        float rho = m / (vc + vs);
        float mc = rho * vc, ms = rho * vs;
        float izz = mc * r * r / 2.0f + ms * 2.0f * r * r / 5.0f;
        float ixx = mc * (L * L / 12.0f + r * r / 4.0f) + ms * (2.0f * r * r / 5.0f + L * L / 4.0f + 3.0f * L * r / 8.0f);
        I[0] = ixx; I[1] = ixx; I[2] = izz;
    }
}
// Rotation matrix (row-major) of a quaternion (w, x, y, z), float32.
template <class F> void quat_matrix(const F* q, F R[3][3]) {
    const F w = q[0], x = q[1], y = q[2], z = q[3];
    F xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
    R[0][0] = F(1) - F(2) * (yy + zz); R[0][1] = F(2) * (xy - wz);        R[0][2] = F(2) * (xz + wy);
    R[1][0] = F(2) * (xy + wz);        R[1][1] = F(1) - F(2) * (xx + zz); R[1][2] = F(2) * (yz - wx);
    R[2][0] = F(2) * (xz - wy);        R[2][1] = F(2) * (yz + wx);        R[2][2] = F(1) - F(2) * (xx + yy);
}
// Compound volume and principal moments (float32): the parts share the mass by volume; each
// part's moments are rotated into the body frame and moved to the origin (parallel axes), summed
// in part order; the diagonal is the body's principal moments.
float compound_volume(const ms_compound_desc& c) {
    float v = 0.0f;
    for (int k = 0; k < c.n_children; ++k) v = v + prim_volume(c.shape[k], c.dims[k]);
    return v;
}
void compound_inertia(const ms_compound_desc& c, float m, float I[3]) {
    const float vt = compound_volume(c);
    I[0] = I[1] = I[2] = 0.0f;
    for (int k = 0; k < c.n_children; ++k) {
        const float mk = m * (prim_volume(c.shape[k], c.dims[k]) / vt);
        float Ik[3];
        prim_inertia(c.shape[k], c.dims[k], mk, Ik);
        float R[3][3];
        quat_matrix(c.pose[k] + 3, R);
        const float* cc = c.pose[k];
        const float c2 = cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2];
        for (int i = 0; i < 3; ++i) {
            const float rot = R[i][0] * Ik[0] * R[i][0] + R[i][1] * Ik[1] * R[i][1] + R[i][2] * Ik[2] * R[i][2];
            const float par = mk * (c2 - cc[i] * cc[i]);
            I[i] = I[i] + (rot + par);
        }
    }
}

// A compound table entry: 1..4 parts of primitive shape with positive dims, finite poses and
// unit quaternions, built in its principal frame with the centre of mass at the origin (checked
// in float64: centre within 1e-4 of the extent, products of inertia within 1e-3 of the largest
// moment).
ms_status validate_compound(const ms_compound_desc& c, int k) {
    if (c.n_children < 1 || c.n_children > MS_MAX_PARTS)
        return fail(MS_E_INVALID_ARG, "compound %d: %d parts (1..%d supported)", k, c.n_children, MS_MAX_PARTS);
    double vt = 0.0, com[3] = {0, 0, 0}, ext = 0.0;
    for (int j = 0; j < c.n_children; ++j) {
        const int sh = c.shape[j];
        if (sh < MS_SPHERE || sh > MS_BOX) return fail(MS_E_INVALID_ARG, "compound %d part %d: bad shape %d", k, j, sh);
        const int nd = sh == MS_SPHERE ? 1 : (sh == MS_CAPSULE ? 2 : 3);
        for (int r = 0; r < nd; ++r)
            if (!(c.dims[j][r] > 0.0f) || !std::isfinite(c.dims[j][r]))
                return fail(MS_E_INVALID_ARG, "compound %d part %d: dims must be positive", k, j);
        for (int r = 0; r < 7; ++r)
            if (!std::isfinite(c.pose[j][r])) return fail(MS_E_INVALID_ARG, "compound %d part %d: non-finite pose", k, j);
        const float* q = c.pose[j] + 3;
        const double qn = double(q[0]) * q[0] + double(q[1]) * q[1] + double(q[2]) * q[2] + double(q[3]) * q[3];
        if (std::fabs(qn - 1.0) > 2e-5) return fail(MS_E_INVALID_ARG, "compound %d part %d: quaternion not unit", k, j);
        const double v = prim_volume(sh, c.dims[j]);
        vt += v;
        double bound = sh == MS_SPHERE ? c.dims[j][0]
                     : sh == MS_CAPSULE ? double(c.dims[j][0]) + c.dims[j][1]
                                        : std::sqrt(double(c.dims[j][0]) * c.dims[j][0] + double(c.dims[j][1]) * c.dims[j][1] +
                                                    double(c.dims[j][2]) * c.dims[j][2]);
        double cn = 0.0;
        for (int r = 0; r < 3; ++r) { com[r] += v * c.pose[j][r]; cn += double(c.pose[j][r]) * c.pose[j][r]; }
        ext = std::max(ext, std::sqrt(cn) + bound);
    }
    for (int r = 0; r < 3; ++r)
        if (std::fabs(com[r] / vt) > 1e-4 * ext)
            return fail(MS_E_INVALID_ARG, "compound %d: centre of mass not at the body origin", k);
    // full inertia tensor (unit mass) in float64
    double T[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < c.n_children; ++j) {
        const double mj = prim_volume(c.shape[j], c.dims[j]) / vt;
        float Ik[3];
        prim_inertia(c.shape[j], c.dims[j], float(mj), Ik);
        double q[4] = {c.pose[j][3], c.pose[j][4], c.pose[j][5], c.pose[j][6]};
        double R[3][3];
        quat_matrix(q, R);
        const double cc[3] = {c.pose[j][0], c.pose[j][1], c.pose[j][2]};
        const double c2 = cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2];
        for (int a = 0; a < 3; ++a)
            for (int b2 = 0; b2 < 3; ++b2)
                T[a][b2] += R[a][0] * Ik[0] * R[b2][0] + R[a][1] * Ik[1] * R[b2][1] + R[a][2] * Ik[2] * R[b2][2] +
                            mj * ((a == b2 ? c2 : 0.0) - cc[a] * cc[b2]);
    }
    const double dmax = std::max(T[0][0], std::max(T[1][1], T[2][2]));
    if (std::fabs(T[0][1]) > 1e-3 * dmax || std::fabs(T[0][2]) > 1e-3 * dmax || std::fabs(T[1][2]) > 1e-3 * dmax)
        return fail(MS_E_INVALID_ARG, "compound %d: the body axes are not its principal axes", k);
    return MS_OK;
}

ms_status validate(const ms_sim_params* p, const ms_scene_desc* s) {
    if (!p || !s) return fail(MS_E_INVALID_ARG, "null params or scene");
    if (s->n_envs <= 0) return fail(MS_E_INVALID_ARG, "n_envs must be positive (got %d)", s->n_envs);
    if (!s->env_body_off || !s->env_joint_off || !s->bodies) return fail(MS_E_INVALID_ARG, "null scene arrays");
    if (!(p->dt > 0.0f) || !std::isfinite(p->dt)) return fail(MS_E_INVALID_ARG, "dt must be positive");
    if (p->pos_iters < 1 || p->pos_iters > 256) return fail(MS_E_INVALID_ARG, "pos_iters out of range [1, 256]");
    if (p->vel_iters < 0 || p->vel_iters > 256) return fail(MS_E_INVALID_ARG, "vel_iters out of range [0, 256]");
    if (p->solver != MS_SOLVER_TGS && p->solver != MS_SOLVER_PGS) return fail(MS_E_INVALID_ARG, "unknown solver");
    if (p->joint_iters < 0 || p->joint_iters > 64) return fail(MS_E_INVALID_ARG, "joint_iters out of range [0, 64]");
    if (p->warm_start && !(std::isfinite(p->warm_radius) && p->warm_radius >= 0.0f))
        return fail(MS_E_INVALID_ARG, "warm_radius must be finite and >= 0");
    if (s->env_body_off[0] != 0 || s->env_joint_off[0] != 0) return fail(MS_E_INVALID_ARG, "offsets must start at 0");
    if (s->n_compounds < 0 || (s->n_compounds > 0 && !s->compounds))
        return fail(MS_E_INVALID_ARG, "bad compound table (%d entries)", s->n_compounds);
    for (int k = 0; k < s->n_compounds; ++k)
        if (ms_status st = validate_compound(s->compounds[k], k); st != MS_OK) return st;
    for (int e = 0; e < s->n_envs; ++e) {
        int nb = s->env_body_off[e + 1] - s->env_body_off[e];
        int nj = s->env_joint_off[e + 1] - s->env_joint_off[e];
        if (nb < 1 || nb > MS_MAX_BODIES_PER_ENV)
            return fail(MS_E_CAPACITY, "env %d has %d bodies (1..%d supported)", e, nb, MS_MAX_BODIES_PER_ENV);
        if (nj < 0 || nj > MS_MAX_JOINTS_PER_ENV)
            return fail(MS_E_CAPACITY, "env %d has %d joints (0..%d supported)", e, nj, MS_MAX_JOINTS_PER_ENV);
        if (nj > 0 && !s->joints) return fail(MS_E_INVALID_ARG, "null joints array");
        {
            // solver blocks (joints + manifolds) of one env: the one-env warm-start lists hold
            // their headers in 4 registers of 64 lanes
            int n_dyn = 0;
            for (int i = 0; i < nb; ++i) n_dyn += (s->bodies[s->env_body_off[e] + i].flags & MS_BODY_STATIC) ? 0 : 1;
            const int mcap = p->max_manifolds_per_env > 0 ? p->max_manifolds_per_env : std::min(3 * n_dyn + 4, 192);
            if (nj + mcap > MS_MAX_BLOCKS_PER_ENV)
                return fail(MS_E_CAPACITY, "env %d: %d joints + %d manifolds exceed %d solver blocks per env", e, nj, mcap,
                            MS_MAX_BLOCKS_PER_ENV);
        }
        for (int i = 0; i < nb; ++i) {
            const ms_body_desc& b = s->bodies[s->env_body_off[e] + i];
            if (b.shape < MS_SPHERE || b.shape > MS_COMPOUND) return fail(MS_E_INVALID_ARG, "env %d body %d: bad shape", e, i);
            if ((b.flags & ~MS_BODY_STATIC) != 0) return fail(MS_E_INVALID_ARG, "env %d body %d: bad flags", e, i);
            if (b.shape == MS_COMPOUND) {
                const float ci = b.dims[0];
                if (!(ci >= 0.0f) || !(ci < float(s->n_compounds)) || ci != float(int(ci)))
                    return fail(MS_E_INVALID_ARG, "env %d body %d: compound index %g outside the table of %d", e, i,
                                double(ci), s->n_compounds);
                if (!(b.flags & MS_BODY_STATIC) && !(b.mass > 0.0f) && !(b.density > 0.0f))
                    return fail(MS_E_INVALID_ARG, "env %d body %d: dynamic body needs mass or density", e, i);
                continue;
            }
            int nd = b.shape == MS_SPHERE ? 1 : (b.shape == MS_CAPSULE ? 2 : 3);
            for (int k = 0; k < nd; ++k)
                if (!(b.dims[k] > 0.0f) || !std::isfinite(b.dims[k]))
                    return fail(MS_E_INVALID_ARG, "env %d body %d: dims must be positive", e, i);
            if (b.shape == MS_CAPSULE && b.dims[1] < 0.0f) return fail(MS_E_INVALID_ARG, "bad capsule");
            if (!(b.flags & MS_BODY_STATIC) && !(b.mass > 0.0f) && !(b.density > 0.0f))
                return fail(MS_E_INVALID_ARG, "env %d body %d: dynamic body needs mass or density", e, i);
        }
        for (int j = 0; j < nj; ++j) {
            const ms_joint_desc& d = s->joints[s->env_joint_off[e] + j];
            if (d.parent < -1 || d.parent >= nb || d.child < 0 || d.child >= nb || d.parent == d.child)
                return fail(MS_E_INVALID_ARG, "env %d joint %d: bad body index", e, j);
            if (s->bodies[s->env_body_off[e] + d.child].flags & MS_BODY_STATIC)
                return fail(MS_E_INVALID_ARG, "env %d joint %d: child must be dynamic", e, j);
            if (!std::isfinite(d.target) || !std::isfinite(d.kp) || !std::isfinite(d.kd) || d.kp < 0 || d.kd < 0)
                return fail(MS_E_INVALID_ARG, "env %d joint %d: kp, kd must be finite and >= 0, target finite", e, j);
            if (d.type != MS_JOINT_REVOLUTE && d.type != MS_JOINT_PRISMATIC)
                return fail(MS_E_INVALID_ARG, "env %d joint %d: unknown joint type %d", e, j, d.type);
            if (d.limited) {
                const float lim = d.type == MS_JOINT_REVOLUTE ? 3.14159265f : 1e30f;
                if (!std::isfinite(d.lower) || !std::isfinite(d.upper) || !(d.lower <= d.upper) || d.lower < -lim ||
                    d.upper > lim)
                    return fail(MS_E_INVALID_ARG, "env %d joint %d: limits need finite lower <= upper (within "
                                "[-pi, pi] for a revolute joint)", e, j);
            }
        }
    }
    return MS_OK;
}


// Bins for the single-launch form: tiles (sorted by LDS need, largest first) placed first-fit
// into bins of at most BIN_WAVES tiles and BIN_BUDGET words.  Only for batches with more than
// one LDS class; otherwise the class launch is already a single launch.
template <class TileRef, class BinVec, class IntVec>
int pack_bins(int n_tiles, TileRef tile_ref, BinVec& bins, IntVec& used, int max_tiles = BIN_WAVES,
              int budget = BIN_BUDGET) {
    bins.clear();
    used.clear();
    int bin_words = 0;
    for (int t = 0; t < n_tiles; ++t) {
        const int w = tile_ref(t).lds_words;
        int k = 0;
        while (k < int(bins.size()) && (bins[k].count == max_tiles || used[k] + w > budget)) ++k;
        if (k == int(bins.size())) {
            bins.push_back(Bin{});
            used.push_back(0);
        }
        Bin& bn = bins[k];
        bn.tile[bn.count] = t;
        bn.off[bn.count] = used[k];
        bn.count++;
        used[k] += w;
        bin_words = std::max(bin_words, used[k]);
    }
    return bin_words;
}
void make_bins(Plan& out) {
    out.bins.clear();
    out.bin_words = 0;
    if (out.classes.size() < 2 || out.launch_mode == 1) return;
    std::vector<int> used;
    out.bin_words = pack_bins(int(out.tiles.size()), [&](int t) -> const Tile& { return out.tiles[t]; }, out.bins, used,
                              out.bin_tiles, out.bin_budget);
    // bins in order of their longest tile's estimated work (the waves of a bin run side by side),
    // largest first, for the same reason as the tiles
    std::vector<float> bcost(out.bins.size(), 0.0f);
    for (size_t k = 0; k < out.bins.size(); ++k)
        for (int w = 0; w < out.bins[k].count; ++w) {
            const Tile& t = out.tiles[out.bins[k].tile[w]];
            float c = 0.0f;
            for (int e = 0; e < t.count; ++e) c += out.info[out.tenv[t.first + e].env].cost;
            bcost[k] = std::max(bcost[k], c);
        }
    std::vector<int> idx(out.bins.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = int(k);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return bcost[x] > bcost[y]; });
    std::vector<Bin> sorted(out.bins.size());
    for (size_t k = 0; k < idx.size(); ++k) sorted[k] = out.bins[idx[k]];
    out.bins.swap(sorted);
}

constexpr int TILE_BUDGET = 10240;  // tile LDS budget in words (40 KiB: four tiles per CU) unless one env needs more

// Tiles, env slots and LDS classes from the per-env sizes and lanes (info[e].lanes): envs sorted
// by (lanes, LDS words) when packing, consecutive envs of equal lanes share a tile while it fits.
void make_tiles(Plan& out, bool pack) {
    const int E = int(out.info.size());
    std::vector<int> order(E);
    for (int e = 0; e < E; ++e) order[e] = e;
    if (pack)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (out.info[a].lanes != out.info[b].lanes) return out.info[a].lanes < out.info[b].lanes;
            return out.info[a].words < out.info[b].words;
        });
    out.tiles.clear();
    out.tenv.clear();
    out.max_tile_words = 0;
    Tile cur{0, 0, 0, 0};
    for (int k = 0; k < E; ++k) {
        int e = order[k];
        const EnvInfo& I = out.info[e];
        bool fits = cur.count > 0 && cur.lanes == I.lanes && cur.count < WAVE / I.lanes &&
                    cur.lds_words + I.words <= std::max(TILE_BUDGET, I.words);
        if (!fits) {
            if (cur.count > 0) out.tiles.push_back(cur);
            cur = Tile{int(out.tenv.size()), 0, I.lanes, 0};
        }
        out.tenv.push_back(TileEnv{0, e, cur.lds_words, I.n, I.nj, I.cap, I.mcap, 0});
        cur.lds_words += I.words;
        cur.count++;
    }
    if (cur.count > 0) out.tiles.push_back(cur);
    // LDS classes: tiles sorted by LDS need (largest first), then cut (cut_classes).  Among
    // tiles of one LDS size the estimated work decides, largest first: workgroups are handed
    // out in order, so the longest tiles start first and the short ones fill the tail.
    std::vector<float> tcost(out.tiles.size(), 0.0f);
    for (size_t t = 0; t < out.tiles.size(); ++t)
        for (int k = 0; k < out.tiles[t].count; ++k) tcost[t] += out.info[out.tenv[out.tiles[t].first + k].env].cost;
    std::vector<int> idx(out.tiles.size());
    for (size_t t = 0; t < idx.size(); ++t) idx[t] = int(t);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        if (out.tiles[a].lds_words != out.tiles[b].lds_words) return out.tiles[a].lds_words > out.tiles[b].lds_words;
        return tcost[a] > tcost[b];
    });
    std::vector<Tile> sorted(out.tiles.size());
    for (size_t t = 0; t < idx.size(); ++t) sorted[t] = out.tiles[idx[t]];
    out.tiles.swap(sorted);
    cut_classes(int(out.tiles.size()), [&](int t) -> Tile& { return out.tiles[t]; }, pack, out.classes);
    for (const Tile& t : out.tiles) out.max_tile_words = std::max(out.max_tile_words, t.lds_words);
    make_bins(out);
}

void plan_batch(const ms_sim_params* p, const ms_scene_desc* s, const ms_plan* plan, Plan& out) {
    const int E = s->n_envs;
    const int forced = plan ? plan->lanes_per_env : 0;
    const bool pack = plan ? plan->pack != 0 : true;
    out.launch_mode = plan ? plan->launch_mode : 0;
    out.info.resize(E);
    for (int e = 0; e < E; ++e) {
        EnvInfo& I = out.info[e];
        I.n = s->env_body_off[e + 1] - s->env_body_off[e];
        I.nj = s->env_joint_off[e + 1] - s->env_joint_off[e];
        I.n_dyn = 0;
        for (int i = 0; i < I.n; ++i) I.n_dyn += (s->bodies[s->env_body_off[e] + i].flags & MS_BODY_STATIC) ? 0 : 1;
        I.cap = p->max_contacts_per_env > 0 ? p->max_contacts_per_env : std::min(6 * I.n_dyn + 8, 384);
        I.mcap = p->max_manifolds_per_env > 0 ? p->max_manifolds_per_env : std::min(3 * I.n_dyn + 4, 192);
        I.words = env_lds_words(I.n, I.nj, I.cap, I.mcap);
        I.lanes = pick_lanes(I, forced, TILE_BUDGET);
        // work estimate: narrowphase and solver cost grow with the bodies' shapes (a box more
        // than a sphere, a compound by its parts) and with the joints
        I.cost = 6.0f * float(I.nj);
        for (int i = 0; i < I.n; ++i) {
            const ms_body_desc& bd = s->bodies[s->env_body_off[e] + i];
            auto shape_cost = [](int sh) { return sh == MS_BOX ? 6.0f : (sh == MS_CAPSULE ? 2.0f : 1.0f); };
            float c = 0.0f;
            if (bd.shape == MS_COMPOUND) {
                const ms_compound_desc& cd = s->compounds[int(bd.dims[0])];
                for (int k = 0; k < cd.n_children; ++k) c += 1.5f * shape_cost(cd.shape[k]);
            } else {
                c = shape_cost(bd.shape);
            }
            I.cost += (bd.flags & MS_BODY_STATIC) ? 0.5f * c : c;
        }
    }
    make_tiles(out, pack);
    out.dbg_pair_off.assign(E + 1, 0);
    out.dbg_pt_off.assign(E + 1, 0);
    out.dbg_man_off.assign(E + 1, 0);
    for (int e = 0; e < E; ++e) {
        const EnvInfo& I = out.info[e];
        out.dbg_pair_off[e + 1] = out.dbg_pair_off[e] + I.n * (I.n + 1) / 2;
        out.dbg_pt_off[e + 1] = out.dbg_pt_off[e] + I.cap;
        out.dbg_man_off[e + 1] = out.dbg_man_off[e] + I.mcap;
    }
}

WsLayout layout_ws(const ms_sim_params* p, const ms_scene_desc* s, const Plan& pl) {
    WsLayout L{};
    const size_t E = size_t(s->n_envs), B = size_t(s->env_body_off[s->n_envs]), J = size_t(s->env_joint_off[s->n_envs]);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + std::max<size_t>(bytes, 4)); return r; };
    L.pos = take(3 * B * 4); L.quat = take(4 * B * 4); L.vel = take(3 * B * 4); L.angvel = take(3 * B * 4);
    L.ipos = take(3 * B * 4); L.iquat = take(4 * B * 4); L.ivel = take(3 * B * 4); L.iang = take(3 * B * 4);
    L.save = take(13 * B * 4 + E * 4);
    L.status = take(E * 4);
    L.bpar = take(3 * B * 16);
    L.body_off = take((E + 1) * 4);
    L.joint_off = take((E + 1) * 4);
    L.jrec = take(J * JREC * 4);
    L.targets = take(J * 4);
    L.tiles = take(E * sizeof(Tile));   // room for any tiling (one env per tile at most)
    L.bins = take(E * sizeof(Bin));     // and for its bins
    L.tenv = take(pl.tenv.size() * sizeof(TileEnv));
    L.bd = take(sizeof(BatchDev));
    L.stats = take(E * NSTAT * 8);
    L.forces = take(3 * B * 4);
    L.bad_ids = take(4);
    L.phase_clock = take(16 * 8);
    L.comp = take(size_t(std::max(s->n_compounds, 0)) * COMP_WORDS * 4);
    if (p->warm_start) {
        // contact cache: header [E][2], manifold records [sum mcap][6], point records [sum cap][4],
        // and a copy of all three for the tuner's save / restore
        const size_t hdr = E * 8, man = size_t(pl.dbg_man_off[E]) * CM_WORDS * 4, pt = size_t(pl.dbg_pt_off[E]) * CP_WORDS * 4;
        L.cache_hdr = take(hdr);
        L.cache_man = take(man);
        L.cache_pt = take(pt);
        L.cache_man_off = take((E + 1) * 4);
        L.cache_pt_off = take((E + 1) * 4);
        L.cache_bytes = L.cache_man_off - L.cache_hdr;   // hdr + man + pt sections, contiguous
        L.cache_save = take(L.cache_bytes);
    }
    if (p->debug_export) {
        L.dbg_pairs = take(size_t(pl.dbg_pair_off[E]) * 16);
        L.dbg_pair_off = take((E + 1) * 4);
        L.dbg_pts = take(size_t(pl.dbg_pt_off[E]) * 32);
        L.dbg_pt_off = take((E + 1) * 4);
        L.dbg_man = take(size_t(pl.dbg_man_off[E]) * 32);
        L.dbg_man_off = take((E + 1) * 4);
        L.dbg_counts = take(E * 16);
    }
    L.total = o;
    return L;
}

// Mass properties (uniform density; centre of mass at the shape centre, or at the origin of a
// compound's body frame).
void mass_props(const ms_body_desc& b, const ms_compound_desc* comps, float& invm, float inv_inertia[3]) {
    if (b.flags & MS_BODY_STATIC) { invm = 0.0f; inv_inertia[0] = inv_inertia[1] = inv_inertia[2] = 0.0f; return; }
    if (b.shape == MS_COMPOUND) {
        const ms_compound_desc& c = comps[int(b.dims[0])];
        const float m = b.mass > 0.0f ? b.mass : b.density * compound_volume(c);
        float I[3];
        compound_inertia(c, m, I);
        invm = 1.0f / m;
        for (int k = 0; k < 3; ++k) inv_inertia[k] = 1.0f / I[k];
        return;
    }
    // float32 throughout, in the order of the step model's definition (uniform density).
    float m;
    if (b.mass > 0.0f) m = b.mass;
    else {
        float fd0 = b.dims[0], fd1 = b.dims[1], fd2 = b.dims[2];
        const float fpi = 3.14159265358979323846f;
        float fv;
        if (b.shape == MS_SPHERE) fv = 4.0f / 3.0f * fpi * fd0 * fd0 * fd0;
        else if (b.shape == MS_CAPSULE) { float L = 2.0f * fd1; fv = fpi * fd0 * fd0 * L + 4.0f / 3.0f * fpi * fd0 * fd0 * fd0; }
        else fv = 8.0f * fd0 * fd1 * fd2;
        m = b.density * fv;
    }
    float I[3];
    float f0 = b.dims[0], f1 = b.dims[1], f2 = b.dims[2];
    if (b.shape == MS_SPHERE) { float i = 2.0f / 5.0f * m * f0 * f0; I[0] = I[1] = I[2] = i; }
    else if (b.shape == MS_BOX) {
        float a = 2.0f * f0, bb = 2.0f * f1, c = 2.0f * f2;
        I[0] = m / 12.0f * (bb * bb + c * c); I[1] = m / 12.0f * (a * a + c * c); I[2] = m / 12.0f * (a * a + bb * bb);
    } else {
        const float fpi = 3.14159265358979323846f;
        float r = f0, L = 2.0f * f1;
        float vc = fpi * r * r * L, vs = 4.0f / 3.0f * fpi * r * r * r;
        float rho = m / (vc + vs);
        float mc = rho * vc, ms = rho * vs;
        float izz = mc * r * r / 2.0f + ms * 2.0f * r * r / 5.0f;
        float ixx = mc * (L * L / 12.0f + r * r / 4.0f) + ms * (2.0f * r * r / 5.0f + L * L / 4.0f + 3.0f * L * r / 8.0f);
        I[0] = ixx; I[1] = ixx; I[2] = izz;
    }
    invm = 1.0f / m;
    for (int k = 0; k < 3; ++k) inv_inertia[k] = 1.0f / I[k];
}

}  // namespace

struct ms_batch {
    ms_sim_params P;
    int E = 0, B = 0, J = 0;
    std::vector<int> body_off, joint_off;
    Plan plan;
    WsLayout lay;
    char* ws = nullptr;
    BatchDev hbd;
    BatchDev* dbd = nullptr;
    int device = 0;
    int grid = 0;
    size_t lds_bytes = 0;
    bool pack = true;
    int max_resident_groups = 0;
    // bumped whenever the tiles, bins or their launch geometry are rewritten (retile); a graph
    // captured under another generation would replay stale launch geometry
    uint64_t plan_gen = 0;
    // every env's joints are ordered parents first (a joint's parent is posed by an earlier
    // joint or by no joint), as the randomised reset's forward kinematics requires
    bool joints_ordered = true;
    // the step accumulates per-body contact forces (ms_set_contact_forces)
    bool forces_on = false;
    // entries of the compound table (compound bodies run in the kernel twins with the optional
    // phases, which hold the compound narrowphase)
    int n_comp = 0;
    // fork / join streams for LDS classes after the first (default priority)
    hipStream_t side[MAX_CLASSES] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[MAX_CLASSES] = {};
    ~ms_batch() {
        for (int k = 0; k < MAX_CLASSES; ++k) {
            if (side[k]) (void)hipStreamDestroy(side[k]);
            if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
    }
};

// Feature level of the kernels a batch runs: 1 with the optional phases (contact forces or
// contact cache on), 3 with compound bodies (a superset), else 0.
static int batch_opt(const ms_batch* b) {
    return b->n_comp > 0 ? 3 : ((b->forces_on || b->P.warm_start != 0) ? 1 : 0);
}

namespace {
template <class T> T* at(char* base, size_t off) { return reinterpret_cast<T*>(base + off); }

void fill_batchdev(ms_batch* b) {
    BatchDev& d = b->hbd;
    std::memset(&d, 0, sizeof(d));
    char* w = b->ws;
    const WsLayout& L = b->lay;
    d.pos = at<float>(w, L.pos); d.quat = at<float>(w, L.quat); d.vel = at<float>(w, L.vel); d.angvel = at<float>(w, L.angvel);
    d.status = at<int>(w, L.status);
    d.bpar = at<float4>(w, L.bpar);
    d.body_off = at<int>(w, L.body_off); d.joint_off = at<int>(w, L.joint_off);
    d.jrec = at<float>(w, L.jrec); d.targets = at<float>(w, L.targets);
    d.B = b->B; d.E = b->E; d.J = b->J;
    const ms_sim_params& p = b->P;
    d.dt = p.dt; d.gx = p.gravity[0]; d.gy = p.gravity[1]; d.gz = p.gravity[2];
    bool tgs = p.solver == MS_SOLVER_TGS;
    d.S = tgs ? std::max(p.pos_iters, 1) : 1;
    d.K = tgs ? 1 : std::max(p.pos_iters, 1);
    d.V = p.vel_iters;
    d.JI = std::max(p.joint_iters, 1);
    d.plane_z = p.plane_z; d.plane_mu = p.plane_friction; d.plane_e = p.plane_restitution; d.delta = p.contact_offset;
    d.plane = p.plane_enabled ? 1 : 0;
    d.beta = p.baumgarte; d.max_depen = p.max_depen_vel; d.beta_j = p.joint_baumgarte; d.bounce = p.bounce_threshold;
    d.lin_damp = p.lin_damping; d.ang_damp = p.ang_damping;
    d.stats = at<long long>(w, L.stats);
    d.bad_ids = at<int>(w, L.bad_ids);
    d.phase_clock = at<unsigned long long>(w, L.phase_clock);
    if (p.warm_start) {
        d.cache_hdr = at<int>(w, L.cache_hdr);
        d.cache_man = at<float>(w, L.cache_man);
        d.cache_man_off = at<int>(w, L.cache_man_off);
        d.cache_pt = at<float>(w, L.cache_pt);
        d.cache_pt_off = at<int>(w, L.cache_pt_off);
        d.warm_radius = p.warm_radius;
    }
    d.forces = b->forces_on ? at<float>(w, L.forces) : nullptr;
    d.comp = b->n_comp > 0 ? at<float>(w, L.comp) : nullptr;
    d.n_comp = b->n_comp;
    if (p.debug_export) {
        d.dbg_pairs = at<int>(w, L.dbg_pairs); d.dbg_pair_off = at<int>(w, L.dbg_pair_off);
        d.dbg_pts = at<float>(w, L.dbg_pts); d.dbg_pt_off = at<int>(w, L.dbg_pt_off);
        d.dbg_man = at<float>(w, L.dbg_man); d.dbg_man_off = at<int>(w, L.dbg_man_off);
        d.dbg_counts = at<int>(w, L.dbg_counts);
    }
}
}  // namespace

extern "C" {

const char* ms_last_error(void) { return g_err.c_str(); }
const char* ms_version(void) { return "libms 0.1 (gfx950)"; }

// Host-side consistency check of the kernel indexing (no device needed): every LDS array of the
// env layout lies inside its allocation and the pair decode enumerates exactly the canonical
// order (a, b), a < b <= n, for every supported body count.  Returns 0 when consistent.
int ms_selfcheck(void) {
    for (int n = 1; n <= MAX_BODIES; ++n) {
        const int P = n * (n + 1) / 2;
        int k = 0;
        for (int a = 0; a < n; ++a)
            for (int b = a + 1; b <= n; ++b, ++k) {
                int pa, pb;
                pair_of(k, n, pa, pb);
                if (pa != a || pb != b) return 1;
            }
        if (k != P) return 2;
        for (int nj = 0; nj <= MAX_JOINTS; nj += 7)
            for (int cap = 1; cap <= 512; cap = cap * 2 + 1)
                for (int mcap = 1; mcap <= cap; mcap = mcap * 2 + 1) {
                    Lay L = make_lay(n, nj, cap, mcap);
                    // every region at least as large as the kernel's use of it, in order, no overlap
                    // (the candidate area later holds the per-body block lists):
                    // contact rows 14 words per point, manifold rows 23 per manifold, schedules of
                    // up to nj + mcap + 66 entries (the joint schedule holds the 65 colouring
                    // cursors when there are no joints)
                    const int start[] = {L.JM, L.JNT, L.JINV, L.CAND, L.PT, L.MAN, L.BCOL, L.ORDER, L.SCHED,
                                         L.JSCHED, L.CSTART, L.SCAL};
                    const int size[] = {2 * n, 31 * nj, 40 * nj, std::max((P + 1) / 2, n + 1 + nj + mcap), 14 * cap, 23 * mcap, (nj + mcap + 1) / 2,
                                        (nj + mcap + 1) / 2, nj + mcap + 66, nj > 0 ? nj + mcap + 66 : N_COLOURS + 1,
                                        N_COLOURS + 2, 32};
                    for (int r = 0; r < 12; ++r) {
                        const int next = r + 1 < 12 ? start[r + 1] : L.total;
                        if (start[r] + size[r] > next) return 3;
                    }
                    if (L.SCAL + 32 > L.total || (L.total & 3)) return 4;
                }
    }
    // bin packing: every tile in exactly one bin slot, at most BIN_WAVES per bin, tile regions
    // disjoint and inside the launch's LDS, which stays within the bin budget
    uint32_t seed = 12345u;
    for (int trial = 0; trial < 64; ++trial) {
        std::vector<Tile> tl(1 + trial * 37 % 1500);
        for (Tile& t : tl) {
            seed = seed * 1664525u + 1013904223u;
            t.lds_words = 4 * int(64 + (seed >> 8) % 4000);   // 1 KiB .. 17 KiB, multiples of 4 words
        }
        std::stable_sort(tl.begin(), tl.end(), [](const Tile& a, const Tile& b) { return a.lds_words > b.lds_words; });
        std::vector<Bin> bins;
        std::vector<int> used;
        const int words = pack_bins(int(tl.size()), [&](int t) -> const Tile& { return tl[t]; }, bins, used);
        if (words > BIN_BUDGET) return 5;
        std::vector<int> seen(tl.size(), 0);
        for (const Bin& bn : bins) {
            if (bn.count < 1 || bn.count > BIN_WAVES) return 6;
            int end = 0;
            for (int k = 0; k < bn.count; ++k) {
                if (bn.tile[k] < 0 || bn.tile[k] >= int(tl.size()) || seen[bn.tile[k]]++) return 7;
                if (bn.off[k] != end || (bn.off[k] & 3)) return 8;
                end += tl[bn.tile[k]].lds_words;
            }
            if (end > words) return 9;
        }
        for (int v : seen)
            if (v != 1) return 10;
    }
    return 0;
}

static ms_status validate_plan(const ms_plan* plan) {
    if (!plan) return MS_OK;
    int g = plan->lanes_per_env;
    if (g != 0 && g != 1 && g != 2 && g != 4 && g != 8 && g != 16 && g != 32 && g != 64)
        return fail(MS_E_INVALID_ARG, "lanes_per_env must be 0 or a power of two <= 64 (got %d)", g);
    if (plan->max_resident_groups < 0) return fail(MS_E_INVALID_ARG, "max_resident_groups must be >= 0");
    return MS_OK;
}

ms_status ms_query_batch_bytes(const ms_sim_params* params, const ms_scene_desc* scene, const ms_plan* plan,
                               size_t* bytes) {
    if (!bytes) return fail(MS_E_INVALID_ARG, "null bytes");
    ms_status st = validate(params, scene);
    if (st == MS_OK) st = validate_plan(plan);
    if (st != MS_OK) return st;
    Plan pl;
    plan_batch(params, scene, plan, pl);
    *bytes = layout_ws(params, scene, pl).total;
    return MS_OK;
}

ms_status ms_create_batch(const ms_sim_params* params, const ms_scene_desc* scene, const ms_plan* plan,
                          void* dev_workspace, size_t ws_bytes, void* hip_stream, ms_batch** out) {
    if (!out) return fail(MS_E_INVALID_ARG, "null out");
    *out = nullptr;
    ms_status st = validate(params, scene);
    if (st == MS_OK) st = validate_plan(plan);
    if (st != MS_OK) return st;
    if (!dev_workspace) return fail(MS_E_INVALID_ARG, "null workspace");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return fail(MS_E_INVALID_ARG, "workspace must be 256-byte aligned");
    ms_batch* b = new ms_batch();
    b->P = *params;
    b->E = scene->n_envs;
    b->B = scene->env_body_off[b->E];
    b->J = scene->env_joint_off[b->E];
    b->body_off.assign(scene->env_body_off, scene->env_body_off + b->E + 1);
    b->joint_off.assign(scene->env_joint_off, scene->env_joint_off + b->E + 1);
    b->n_comp = scene->n_compounds;
    plan_batch(params, scene, plan, b->plan);
    for (int e = 0; e < b->E && b->joints_ordered; ++e) {
        const int n = b->body_off[e + 1] - b->body_off[e];
        std::vector<char> posed(size_t(n), 1);
        for (int j = b->joint_off[e]; j < b->joint_off[e + 1]; ++j) posed[size_t(scene->joints[j].child)] = 0;
        for (int j = b->joint_off[e]; j < b->joint_off[e + 1]; ++j) {
            const ms_joint_desc& d = scene->joints[j];
            if (d.parent >= 0 && !posed[size_t(d.parent)]) { b->joints_ordered = false; break; }
            posed[size_t(d.child)] = 1;
        }
    }
    b->lay = layout_ws(params, scene, b->plan);
    if (ws_bytes < b->lay.total) {
        size_t need = b->lay.total;
        delete b;
        return fail(MS_E_NO_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    }
    b->ws = static_cast<char*>(dev_workspace);
    if (hipGetDevice(&b->device) != hipSuccess) { delete b; return fail(MS_E_DEVICE, "hipGetDevice failed"); }
    fill_batchdev(b);
    b->lds_bytes = size_t(b->plan.max_tile_words) * 4;
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess) max_lds = 65536;
    if (b->lds_bytes > size_t(max_lds)) {
        size_t need = b->lds_bytes;
        delete b;
        return fail(MS_E_CAPACITY, "an env tile needs %zu bytes of LDS; the device allows %d", need, max_lds);
    }
    b->pack = plan ? plan->pack != 0 : true;
    b->max_resident_groups = plan ? plan->max_resident_groups : 0;
    const int n_tiles = int(b->plan.tiles.size());
    b->grid = n_tiles;
    if (b->max_resident_groups > 0) b->grid = std::min(n_tiles, b->max_resident_groups);

    // host staging
    const size_t B = b->B, E = b->E, J = b->J;
    std::vector<float> hs(13 * B);
    std::vector<float4> bp(3 * B);
    for (size_t i = 0; i < B; ++i) {
        const ms_body_desc& d = scene->bodies[i];
        for (int r = 0; r < 3; ++r) hs[r * B + i] = d.pos[r];
        for (int r = 0; r < 4; ++r) hs[3 * B + r * B + i] = d.quat[r];
        for (int r = 0; r < 3; ++r) hs[7 * B + r * B + i] = d.linvel[r];
        for (int r = 0; r < 3; ++r) hs[10 * B + r * B + i] = d.angvel[r];
        float invm, iI[3];
        mass_props(d, scene->compounds, invm, iI);
        int code = d.shape | (d.flags << 8);
        float codef;
        std::memcpy(&codef, &code, 4);
        bp[i] = float4{codef, invm, d.friction, d.restitution};
        bp[B + i] = float4{d.dims[0], d.dims[1], d.dims[2], 0.0f};
        bp[2 * B + i] = float4{iI[0], iI[1], iI[2], 0.0f};
    }
    std::vector<float> jr(std::max<size_t>(J, 1) * JREC);
    std::vector<float> tg(std::max<size_t>(J, 1));
    for (size_t j = 0; j < J; ++j) {
        const ms_joint_desc& d = scene->joints[j];
        float* r = &jr[j * JREC];
        std::memcpy(&r[0], &d.parent, 4);
        std::memcpy(&r[1], &d.child, 4);
        for (int k = 0; k < 3; ++k) r[2 + k] = d.frame_parent[k];
        for (int k = 0; k < 4; ++k) r[5 + k] = d.frame_parent[3 + k];
        for (int k = 0; k < 3; ++k) r[9 + k] = d.frame_child[k];
        for (int k = 0; k < 4; ++k) r[12 + k] = d.frame_child[3 + k];
        r[16] = d.kp;
        r[17] = d.kd;
        const int tl = d.type | (d.limited ? 1 << 8 : 0);
        std::memcpy(&r[18], &tl, 4);
        r[19] = d.limited ? d.lower : 0.0f;
        r[20] = d.limited ? d.upper : 0.0f;
        r[21] = 0.0f;
        tg[j] = d.target;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char* w = b->ws;
    const WsLayout& L = b->lay;
    auto up = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    std::vector<int> zeros(E, 0);
    hipError_t e = hipSuccess;
    const size_t p3 = 3 * B * 4, p4 = 4 * B * 4;
    if (e == hipSuccess) e = up(L.pos, &hs[0], p3);
    if (e == hipSuccess) e = up(L.quat, &hs[3 * B], p4);
    if (e == hipSuccess) e = up(L.vel, &hs[7 * B], p3);
    if (e == hipSuccess) e = up(L.angvel, &hs[10 * B], p3);
    if (e == hipSuccess) e = up(L.ipos, &hs[0], p3);
    if (e == hipSuccess) e = up(L.iquat, &hs[3 * B], p4);
    if (e == hipSuccess) e = up(L.ivel, &hs[7 * B], p3);
    if (e == hipSuccess) e = up(L.iang, &hs[10 * B], p3);
    if (e == hipSuccess) e = up(L.status, zeros.data(), E * 4);
    std::vector<long long> zstats(E * NSTAT, 0);
    if (e == hipSuccess) e = up(L.stats, zstats.data(), E * NSTAT * 8);
    std::vector<float> zforces(3 * B + 1, 0.0f);
    if (e == hipSuccess) e = up(L.forces, zforces.data(), 3 * B * 4);
    if (e == hipSuccess) e = up(L.bad_ids, zforces.data(), 4);
    if (e == hipSuccess) e = up(L.phase_clock, zforces.data(), 16 * 8);
    if (params->warm_start) {
        std::vector<int> zh(2 * E, 0);
        if (e == hipSuccess) e = up(L.cache_hdr, zh.data(), 2 * E * 4);
        if (e == hipSuccess) e = up(L.cache_man_off, b->plan.dbg_man_off.data(), (E + 1) * 4);
        if (e == hipSuccess) e = up(L.cache_pt_off, b->plan.dbg_pt_off.data(), (E + 1) * 4);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e == hipSuccess) e = up(L.bpar, bp.data(), 3 * B * 16);
    std::vector<float> ct(size_t(b->n_comp) * COMP_WORDS, 0.0f);
    for (int k = 0; k < b->n_comp; ++k) {
        const ms_compound_desc& c = scene->compounds[k];
        float* r = &ct[size_t(k) * COMP_WORDS];
        std::memcpy(&r[0], &c.n_children, 4);
        for (int j = 0; j < c.n_children; ++j) {
            float* q = r + 4 + 12 * j;
            std::memcpy(&q[0], &c.shape[j], 4);
            for (int t = 0; t < 3; ++t) q[1 + t] = c.dims[j][t];
            for (int t = 0; t < 7; ++t) q[4 + t] = c.pose[j][t];
        }
    }
    if (e == hipSuccess) e = up(L.comp, ct.data(), ct.size() * 4);
    if (e == hipSuccess) e = up(L.body_off, b->body_off.data(), (E + 1) * 4);
    if (e == hipSuccess) e = up(L.joint_off, b->joint_off.data(), (E + 1) * 4);
    if (e == hipSuccess) e = up(L.jrec, jr.data(), J * JREC * 4);
    if (e == hipSuccess) e = up(L.targets, tg.data(), J * 4);
    if (e == hipSuccess) e = up(L.tiles, b->plan.tiles.data(), b->plan.tiles.size() * sizeof(Tile));
    if (e == hipSuccess) e = up(L.tenv, b->plan.tenv.data(), b->plan.tenv.size() * sizeof(TileEnv));
    if (e == hipSuccess && !b->plan.bins.empty()) e = up(L.bins, b->plan.bins.data(), b->plan.bins.size() * sizeof(Bin));
    if (e == hipSuccess) e = up(L.bd, &b->hbd, sizeof(BatchDev));
    if (params->debug_export) {
        if (e == hipSuccess) e = up(L.dbg_pair_off, b->plan.dbg_pair_off.data(), (E + 1) * 4);
        if (e == hipSuccess) e = up(L.dbg_pt_off, b->plan.dbg_pt_off.data(), (E + 1) * 4);
        if (e == hipSuccess) e = up(L.dbg_man_off, b->plan.dbg_man_off.data(), (E + 1) * 4);
        std::vector<int> zc(4 * E, 0);
        if (e == hipSuccess) e = up(L.dbg_counts, zc.data(), 16 * E);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    // the staging vectors go out of scope here: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete b;
        return fail(MS_E_DEVICE, "upload failed: %s", hipGetErrorString(e));
    }
    b->dbd = at<BatchDev>(w, L.bd);
    *out = b;
    return MS_OK;
}

// Side streams and events of the LDS-class fork / join, created once per batch.
static ms_status ensure_side_streams(ms_batch* b) {
    if (b->plan.classes.size() < 2) return MS_OK;
    if (!b->ev_fork) HIP_OK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    for (size_t k = 1; k < b->plan.classes.size(); ++k) {
        if (!b->side[k]) HIP_OK(hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking));
        if (!b->ev_join[k]) HIP_OK(hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming));
    }
    return MS_OK;
}

// Rebuild the tiles for new per-env lanes and upload them (the workspace has room for any
// tiling).  Synchronises `s`.  The result of a step does not depend on the tiling.
static ms_status retile(ms_batch* b, const std::vector<int>& lanes, hipStream_t s) {
    Plan np = b->plan;   // the batch keeps its plan unless the new one is valid
    for (size_t e = 0; e < lanes.size(); ++e) np.info[e].lanes = lanes[e];
    make_tiles(np, b->pack);
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess) max_lds = 65536;
    if (size_t(np.max_tile_words) * 4 > size_t(max_lds))
        return fail(MS_E_CAPACITY, "a tile would need %d bytes of LDS", np.max_tile_words * 4);
    b->plan = std::move(np);
    b->plan_gen++;
    b->lds_bytes = size_t(b->plan.max_tile_words) * 4;
    const int n_tiles = int(b->plan.tiles.size());
    b->grid = b->max_resident_groups > 0 ? std::min(n_tiles, b->max_resident_groups) : n_tiles;
    HIP_OK(hipMemcpyAsync(b->ws + b->lay.tiles, b->plan.tiles.data(), b->plan.tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(b->ws + b->lay.tenv, b->plan.tenv.data(), b->plan.tenv.size() * sizeof(TileEnv),
                          hipMemcpyHostToDevice, s));
    if (!b->plan.bins.empty())
        HIP_OK(hipMemcpyAsync(b->ws + b->lay.bins, b->plan.bins.data(), b->plan.bins.size() * sizeof(Bin),
                              hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return ensure_side_streams(b);
}

ms_status ms_step(ms_batch* b, const float* dev_targets, int32_t n_steps, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (n_steps < 1) return fail(MS_E_INVALID_ARG, "n_steps must be >= 1 (got %d)", n_steps);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (dev_targets && b->J > 0)
        HIP_OK(hipMemcpyAsync(const_cast<float*>(b->hbd.targets), dev_targets, size_t(b->J) * 4, hipMemcpyDeviceToDevice, s));
    const std::vector<LdsClass>& cls = b->plan.classes;
    const Tile* tiles = at<Tile>(b->ws, b->lay.tiles);
    const TileEnv* tenv = at<TileEnv>(b->ws, b->lay.tenv);
    const int grid_cap = b->max_resident_groups;
    const int opt = batch_opt(b);
    if (cls.size() == 1) return launch_class(cls[0], b->dbd, tiles, tenv, int(n_steps), grid_cap, s, opt);
    if (!b->plan.bins.empty()) {   // every tile in one launch, a bin per workgroup
        const int nb = int(b->plan.bins.size());
        hipLaunchKernelGGL(bins_kernel(opt), dim3(nb), dim3(WAVE * BIN_WAVES), size_t(b->plan.bin_words) * 4, s, b->dbd,
                           tiles, at<Bin>(b->ws, b->lay.bins), nb, tenv, int(n_steps));
        HIP_OK(hipGetLastError());
        return MS_OK;
    }
    // one launch per LDS class: the largest class on the caller's stream, the others on side
    // streams forked from and joined back into it
    if (ms_status st = ensure_side_streams(b); st != MS_OK) return st;
    HIP_OK(hipEventRecord(b->ev_fork, s));
    for (size_t k = 0; k < cls.size(); ++k) {
        hipStream_t sk = k == 0 ? s : b->side[k];
        if (k > 0) HIP_OK(hipStreamWaitEvent(sk, b->ev_fork, 0));
        if (ms_status st = launch_class(cls[k], b->dbd, tiles, tenv, int(n_steps), grid_cap, sk, opt); st != MS_OK) return st;
        if (k > 0) {
            HIP_OK(hipEventRecord(b->ev_join[k], sk));
            HIP_OK(hipStreamWaitEvent(s, b->ev_join[k], 0));
        }
    }
    return MS_OK;
}

ms_status ms_reset_envs(ms_batch* b, const int32_t* dev_env_ids, int32_t n_ids, const ms_state_view* src,
                        void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (n_ids < 0) return fail(MS_E_INVALID_ARG, "n_ids must be >= 0");
    if (n_ids == 0) return MS_OK;
    if (!dev_env_ids) return fail(MS_E_INVALID_ARG, "null env ids");
    const float *sp, *sq, *sv, *sw;
    if (src) {
        if (!src->pos || !src->quat || !src->linvel || !src->angvel) return fail(MS_E_INVALID_ARG, "null source plane");
        sp = src->pos; sq = src->quat; sv = src->linvel; sw = src->angvel;
    } else {
        sp = at<float>(b->ws, b->lay.ipos); sq = at<float>(b->ws, b->lay.iquat);
        sv = at<float>(b->ws, b->lay.ivel); sw = at<float>(b->ws, b->lay.iang);
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(ms_reset_kernel, dim3(n_ids), dim3(WAVE), 0, s, b->hbd, dev_env_ids, int(n_ids), sp, sq, sv, sw);
    HIP_OK(hipGetLastError());
    return MS_OK;
}

ms_status ms_reset_envs_random(ms_batch* b, const int32_t* dev_env_ids, int32_t n_ids, const ms_reset_noise* noise,
                               uint64_t seed, uint32_t count, void* hip_stream) {
    if (!b || !noise) return fail(MS_E_INVALID_ARG, "null batch or noise");
    if (n_ids < 0) return fail(MS_E_INVALID_ARG, "n_ids must be >= 0");
    if (n_ids == 0) return MS_OK;
    if (!dev_env_ids) return fail(MS_E_INVALID_ARG, "null env ids");
    const float nzv[3] = {noise->joint_sigma, noise->xy_half, noise->yaw_half};
    for (float v : nzv)
        if (!(std::isfinite(v) && v >= 0.0f)) return fail(MS_E_INVALID_ARG, "noise scales must be finite and >= 0");
    if (!b->joints_ordered)
        return fail(MS_E_INVALID_ARG, "an env's joints are not ordered parents first (forward kinematics needs it)");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    ResetNoiseDev nz{noise->joint_sigma, noise->xy_half, noise->yaw_half, noise->targets_follow ? 1 : 0};
    hipLaunchKernelGGL(ms_reset_random_kernel, dim3((n_ids + 63) / 64), dim3(64), 0, s, b->hbd, dev_env_ids, int(n_ids),
                       at<float>(b->ws, b->lay.ipos), at<float>(b->ws, b->lay.iquat), nz, uint32_t(seed & 0xFFFFFFFFu),
                       uint32_t(seed >> 32), count, b->hbd.bad_ids);
    HIP_OK(hipGetLastError());
    return MS_OK;
}

ms_status ms_apply_actions(ms_batch* b, const float* dev_actions, const float* dev_low, const float* dev_high, float low,
                           float high, void* hip_stream) {
    if (!b || !dev_actions) return fail(MS_E_INVALID_ARG, "null batch or actions");
    if ((!dev_low && !std::isfinite(low)) || (!dev_high && !std::isfinite(high)))
        return fail(MS_E_INVALID_ARG, "scalar bounds must be finite");
    if (b->J == 0) return MS_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(ms_apply_actions_kernel, dim3((b->J + 255) / 256), dim3(256), 0, s, const_cast<float*>(b->hbd.targets),
                       dev_actions, dev_low, dev_high, low, high, b->J);
    HIP_OK(hipGetLastError());
    return MS_OK;
}

ms_status ms_get_targets(ms_batch* b, float* dev_out, void* hip_stream) {
    if (!b || (!dev_out && b->J > 0)) return fail(MS_E_INVALID_ARG, "null batch or output");
    if (b->J == 0) return MS_OK;
    HIP_OK(hipMemcpyAsync(dev_out, b->hbd.targets, size_t(b->J) * 4, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)));
    return MS_OK;
}

ms_status ms_get_joint_positions(ms_batch* b, float* dev_out, void* hip_stream) {
    if (!b || (!dev_out && b->J > 0)) return fail(MS_E_INVALID_ARG, "null batch or output");
    if (b->J == 0) return MS_OK;
    hipLaunchKernelGGL(ms_joint_positions_kernel, dim3((b->E + 63) / 64), dim3(64), 0, static_cast<hipStream_t>(hip_stream),
                       b->hbd, dev_out);
    HIP_OK(hipGetLastError());
    return MS_OK;
}

ms_status ms_set_contact_forces(ms_batch* b, int32_t enable, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (b->forces_on != (enable != 0)) b->plan_gen++;   // the kernel twin changes: captured graphs are stale
    b->forces_on = enable != 0;
    b->hbd.forces = b->forces_on ? at<float>(b->ws, b->lay.forces) : nullptr;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (b->forces_on) HIP_OK(hipMemsetAsync(b->hbd.forces, 0, size_t(b->B) * 12, s));
    // the device copy of the batch record is read by graph replays and the class launches
    HIP_OK(hipMemcpyAsync(b->dbd, &b->hbd, sizeof(BatchDev), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return MS_OK;
}

ms_status ms_get_contact_forces(ms_batch* b, float* dev_out, void* hip_stream) {
    if (!b || !dev_out) return fail(MS_E_INVALID_ARG, "null batch or output");
    if (!b->forces_on) return fail(MS_E_STATE, "contact forces are not enabled (ms_set_contact_forces)");
    HIP_OK(hipMemcpyAsync(dev_out, b->hbd.forces, size_t(b->B) * 12, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)));
    return MS_OK;
}

ms_status ms_get_phase_clocks(ms_batch* b, int64_t* host_cycles, int32_t reset, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
#ifndef MS_PHASE_CLOCK
    (void)host_cycles; (void)reset; (void)hip_stream;
    return fail(MS_E_STATE, "this build has no per-phase clock (build with -DMS_PHASE_CLOCK)");
#else
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    std::vector<int64_t> v(16, 0);
    HIP_OK(hipMemcpyAsync(v.data(), b->hbd.phase_clock, 16 * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (host_cycles) std::copy(v.begin(), v.end(), host_cycles);
    if (reset) {
        std::fill(v.begin(), v.end(), 0);
        HIP_OK(hipMemcpyAsync(b->hbd.phase_clock, v.data(), 16 * 8, hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return MS_OK;
#endif
}

ms_status ms_get_invalid_ids(ms_batch* b, int32_t* host_count, int32_t clear, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int v = 0;
    HIP_OK(hipMemcpyAsync(&v, b->hbd.bad_ids, 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (host_count) *host_count = v;
    if (clear) {
        const int z = 0;
        HIP_OK(hipMemcpyAsync(b->hbd.bad_ids, &z, 4, hipMemcpyHostToDevice, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return MS_OK;
}

ms_status ms_get_state(ms_batch* b, const ms_state_view* dst, void* hip_stream) {
    if (!b || !dst) return fail(MS_E_INVALID_ARG, "null batch or view");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t B = b->B;
    if (dst->pos) HIP_OK(hipMemcpyAsync(dst->pos, b->hbd.pos, 3 * B * 4, hipMemcpyDeviceToDevice, s));
    if (dst->quat) HIP_OK(hipMemcpyAsync(dst->quat, b->hbd.quat, 4 * B * 4, hipMemcpyDeviceToDevice, s));
    if (dst->linvel) HIP_OK(hipMemcpyAsync(dst->linvel, b->hbd.vel, 3 * B * 4, hipMemcpyDeviceToDevice, s));
    if (dst->angvel) HIP_OK(hipMemcpyAsync(dst->angvel, b->hbd.angvel, 3 * B * 4, hipMemcpyDeviceToDevice, s));
    if (dst->status) HIP_OK(hipMemcpyAsync(dst->status, b->hbd.status, size_t(b->E) * 4, hipMemcpyDeviceToDevice, s));
    return MS_OK;
}

ms_status ms_get_layout(ms_batch* b, int32_t* host_env_body_off, int32_t* host_env_joint_off) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (host_env_body_off) std::copy(b->body_off.begin(), b->body_off.end(), host_env_body_off);
    if (host_env_joint_off) std::copy(b->joint_off.begin(), b->joint_off.end(), host_env_joint_off);
    return MS_OK;
}

ms_status ms_get_sizes(ms_batch* b, int32_t* n_envs, int32_t* n_bodies, int32_t* n_joints) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (n_envs) *n_envs = b->E;
    if (n_bodies) *n_bodies = b->B;
    if (n_joints) *n_joints = b->J;
    return MS_OK;
}

ms_status ms_get_classes(ms_batch* b, int32_t* n_classes, int32_t* host_classes) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (n_classes) *n_classes = int(b->plan.classes.size());
    if (host_classes)
        for (size_t k = 0; k < b->plan.classes.size(); ++k) {
            const LdsClass& c = b->plan.classes[k];
            int32_t* o = host_classes + 5 * k;
            o[0] = c.n_tiles; o[1] = c.lds_words * 4; o[2] = c.n_one > 0 ? c.variant : c.variant_gen;
            o[3] = c.lanes; o[4] = c.first_tile;
        }
    return MS_OK;
}

ms_status ms_get_plan(ms_batch* b, int32_t* n_tiles, int32_t* grid, int32_t* lds_bytes, int32_t* host_env_lanes) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    const bool bins = !b->plan.bins.empty();
    if (n_tiles) *n_tiles = int(b->plan.tiles.size());
    if (grid) *grid = bins ? int(b->plan.bins.size()) : b->grid;
    if (lds_bytes) *lds_bytes = bins ? b->plan.bin_words * 4 : int(b->lds_bytes);
    if (host_env_lanes)
        for (int e = 0; e < b->E; ++e) host_env_lanes[e] = b->plan.info[e].lanes;
    return MS_OK;
}

ms_status ms_get_contacts(ms_batch* b, int32_t* host_pairs, int32_t pairs_cap, float* host_points, int32_t points_cap,
                          float* host_manifolds, int32_t manifolds_cap, int32_t* n_pairs, int32_t* n_points,
                          int32_t* n_manifolds, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (!b->P.debug_export) return fail(MS_E_STATE, "contact export needs debug_export in the sim params");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_OK(hipStreamSynchronize(s));
    const int E = b->E;
    const Plan& pl = b->plan;
    std::vector<int> counts(size_t(E) * 4);
    HIP_OK(hipMemcpy(counts.data(), b->hbd.dbg_counts, size_t(E) * 16, hipMemcpyDeviceToHost));
    std::vector<int> dp(size_t(pl.dbg_pair_off[E]) * 4);
    std::vector<float> dpt(size_t(pl.dbg_pt_off[E]) * 8), dm(size_t(pl.dbg_man_off[E]) * 8);
    if (!dp.empty()) HIP_OK(hipMemcpy(dp.data(), b->hbd.dbg_pairs, dp.size() * 4, hipMemcpyDeviceToHost));
    if (!dpt.empty()) HIP_OK(hipMemcpy(dpt.data(), b->hbd.dbg_pts, dpt.size() * 4, hipMemcpyDeviceToHost));
    if (!dm.empty()) HIP_OK(hipMemcpy(dm.data(), b->hbd.dbg_man, dm.size() * 4, hipMemcpyDeviceToHost));
    int np = 0, npt = 0, nm = 0;
    for (int e = 0; e < E; ++e) {
        const EnvInfo& I = pl.info[e];
        int nc = std::min(std::max(counts[4 * e], 0), I.n * (I.n + 1) / 2);
        int nps = std::min(std::max(counts[4 * e + 1], 0), I.cap);
        int nms = std::min(std::max(counts[4 * e + 2], 0), I.mcap);
        for (int k = 0; k < nc; ++k, ++np) {
            if (host_pairs && np < pairs_cap) {
                const int* r = &dp[4 * size_t(pl.dbg_pair_off[e] + k)];
                int32_t* o = host_pairs + 5 * size_t(np);
                o[0] = e; o[1] = r[0]; o[2] = r[1]; o[3] = r[2]; o[4] = r[3];
            }
        }
        for (int k = 0; k < nps; ++k, ++npt) {
            if (host_points && npt < points_cap) {
                const float* r = &dpt[8 * size_t(pl.dbg_pt_off[e] + k)];
                std::copy(r, r + 8, host_points + 8 * size_t(npt));
            }
        }
        for (int k = 0; k < nms; ++k, ++nm) {
            if (host_manifolds && nm < manifolds_cap) {
                const float* r = &dm[8 * size_t(pl.dbg_man_off[e] + k)];
                float* o = host_manifolds + 8 * size_t(nm);
                int pair_idx, colour;
                std::memcpy(&pair_idx, &r[0], 4);
                std::memcpy(&colour, &r[1], 4);
                o[0] = float(e); o[1] = float(pair_idx); o[2] = float(colour);
                o[3] = r[2]; o[4] = r[3]; o[5] = r[4]; o[6] = r[5]; o[7] = r[6];
            }
        }
    }
    if (n_pairs) *n_pairs = np;
    if (n_points) *n_points = npt;
    if (n_manifolds) *n_manifolds = nm;
    return MS_OK;
}

ms_status ms_tune_batch(ms_batch* b, int32_t trial_steps, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    if (trial_steps < 1 || trial_steps > 1000) return fail(MS_E_INVALID_ARG, "trial_steps out of range [1, 1000]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t B = b->B, E = b->E;
    char* w = b->ws;
    const WsLayout& L = b->lay;
    // save the state (and status, stats) so that tuning leaves no trace
    const size_t st_bytes[4] = {3 * B * 4, 4 * B * 4, 3 * B * 4, 3 * B * 4};
    const size_t st_off[4] = {L.pos, L.quat, L.vel, L.angvel};
    size_t o = L.save;
    for (int k = 0; k < 4; ++k) { HIP_OK(hipMemcpyAsync(w + o, w + st_off[k], st_bytes[k], hipMemcpyDeviceToDevice, s)); o += st_bytes[k]; }
    HIP_OK(hipMemcpyAsync(w + o, w + L.status, E * 4, hipMemcpyDeviceToDevice, s));
    if (b->P.warm_start) HIP_OK(hipMemcpyAsync(w + L.cache_save, w + L.cache_hdr, L.cache_bytes, hipMemcpyDeviceToDevice, s));
    std::vector<long long> stats_save(E * NSTAT);
    HIP_OK(hipMemcpyAsync(stats_save.data(), w + L.stats, E * NSTAT * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    auto restore = [&]() -> ms_status {
        size_t oo = L.save;
        for (int k = 0; k < 4; ++k) { HIP_OK(hipMemcpyAsync(w + st_off[k], w + oo, st_bytes[k], hipMemcpyDeviceToDevice, s)); oo += st_bytes[k]; }
        HIP_OK(hipMemcpyAsync(w + L.status, w + oo, E * 4, hipMemcpyDeviceToDevice, s));
        if (b->P.warm_start) HIP_OK(hipMemcpyAsync(w + L.cache_hdr, w + L.cache_save, L.cache_bytes, hipMemcpyDeviceToDevice, s));
        return MS_OK;
    };
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    ms_status st = MS_OK;
    // whole-batch step time of the current plan: restore, one untimed step, trial_steps timed
    auto time_batch = [&](float& ms) -> ms_status {
        if (ms_status r = restore(); r != MS_OK) return r;
        if (ms_status r = ms_step(b, nullptr, 1, s); r != MS_OK) return r;
        HIP_OK(hipEventRecord(e0, s));
        for (int t = 0; t < trial_steps; ++t)
            if (ms_status r = ms_step(b, nullptr, 1, s); r != MS_OK) return r;
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        HIP_OK(hipEventElapsedTime(&ms, e0, e1));
        return MS_OK;
    };
    // 1. lanes per env (64 / lanes envs per wavefront): for each group of envs that the planner
    //    gave the same lanes, try half and twice as many; keep a change only if the whole batch
    //    steps at least 3 % faster
    std::vector<int> orig(E), lanes(E);
    for (size_t e = 0; e < E; ++e) orig[e] = lanes[e] = b->plan.info[e].lanes;
    float best = 0.0f;
    st = time_batch(best);
    std::vector<int> groups(orig);
    std::sort(groups.begin(), groups.end());
    groups.erase(std::unique(groups.begin(), groups.end()), groups.end());
    for (int G : groups) {
        if (st != MS_OK) break;
        for (int alt : {G / 2, G * 2}) {
            if (alt < 1 || alt > WAVE || st != MS_OK) continue;
            std::vector<int> trial(lanes);
            for (size_t e = 0; e < E; ++e)
                if (orig[e] == G) trial[e] = alt;
            if (retile(b, trial, s) != MS_OK) continue;   // e.g. a tile too large: skip this option
            float t = 0.0f;
            st = time_batch(t);
            if (st == MS_OK && t < 0.97f * best) { best = t; lanes = trial; }
        }
        if (st == MS_OK) st = retile(b, lanes, s);
    }
    // 1b. the shape of the bins launch (batches whose tiles need several LDS sizes): at most 2,
    //     3 or 4 tiles per bin in a quarter, a third or half of a CU's LDS (the default is 4 in
    //     half); keep a shape only if the batch steps at least 3 % faster
    if (st == MS_OK && !b->plan.bins.empty()) {
        const int shapes[][2] = {{2, 10240}, {3, 13652}, {4, 13652}, {2, 20480}};
        int best_t = b->plan.bin_tiles, best_b = b->plan.bin_budget;
        for (const auto& sh : shapes) {
            if (st != MS_OK) break;
            b->plan.bin_tiles = sh[0];
            b->plan.bin_budget = sh[1];
            if (retile(b, lanes, s) != MS_OK) continue;
            float t = 0.0f;
            st = time_batch(t);
            if (st == MS_OK && t < 0.97f * best) { best = t; best_t = sh[0]; best_b = sh[1]; }
        }
        b->plan.bin_tiles = best_t;
        b->plan.bin_budget = best_b;
        if (st == MS_OK) st = retile(b, lanes, s);
    }
    // 2. kernel variant per part of each LDS class (one-env part: 2 / 3, general part: 0 / 1),
    //    each part timed alone
    const Tile* tiles = at<Tile>(w, L.tiles);
    const TileEnv* tenv = at<TileEnv>(w, L.tenv);
    // the variants of class launches (a batch run as one launch of bins has fixed builds)
    for (LdsClass& c : b->plan.classes) {
        if (!b->plan.bins.empty()) break;
        for (int part = 0; part < 2 && st == MS_OK; ++part) {
            const int first = part == 0 ? c.first_tile : c.first_tile + c.n_one;
            const int count = part == 0 ? c.n_one : c.n_tiles - c.n_one;
            if (count <= 0) continue;
            float bestc = 1e30f;
            int best_v = part == 0 ? c.variant : c.variant_gen;
            for (int v = part == 0 ? 2 : 0; v < (part == 0 ? 4 : 2) && st == MS_OK; ++v) {
                st = restore();
                if (st != MS_OK) break;
                hipLaunchKernelGGL(kernel_of(v, batch_opt(b)), dim3(count), dim3(WAVE), size_t(c.lds_words) * 4, s, b->dbd,
                                   tiles + first, count, tenv, 1);
                HIP_OK(hipEventRecord(e0, s));
                for (int t = 0; t < trial_steps; ++t)
                    hipLaunchKernelGGL(kernel_of(v, batch_opt(b)), dim3(count), dim3(WAVE), size_t(c.lds_words) * 4,
                                       s, b->dbd, tiles + first, count, tenv, 1);
                HIP_OK(hipGetLastError());
                HIP_OK(hipEventRecord(e1, s));
                HIP_OK(hipEventSynchronize(e1));
                float ms = 0.0f;
                HIP_OK(hipEventElapsedTime(&ms, e0, e1));
                if (ms < bestc) { bestc = ms; best_v = v; }
            }
            (part == 0 ? c.variant : c.variant_gen) = best_v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ms_status rs = restore();
    HIP_OK(hipMemcpyAsync(w + L.stats, stats_save.data(), E * NSTAT * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    return st != MS_OK ? st : rs;
}

ms_status ms_get_stats(ms_batch* b, int64_t* host_stats, int32_t reset, void* hip_stream) {
    if (!b) return fail(MS_E_INVALID_ARG, "null batch");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_OK(hipStreamSynchronize(s));
    const size_t n = size_t(b->E) * NSTAT;
    if (host_stats) {
        std::vector<long long> tmp(n);
        HIP_OK(hipMemcpy(tmp.data(), b->hbd.stats, n * 8, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < n; ++k) host_stats[k] = int64_t(tmp[k]);
    }
    if (reset) {
        std::vector<long long> z(n, 0);
        HIP_OK(hipMemcpy(b->hbd.stats, z.data(), n * 8, hipMemcpyHostToDevice));
    }
    return MS_OK;
}

ms_status ms_destroy_batch(ms_batch* b) {
    delete b;
    return MS_OK;
}

// ----------------------------------------------------------------------------- fused multi-batch step
struct ms_graph {
    ms_batch* b = nullptr;
    uint64_t plan_gen = 0;   // the batch's plan generation at capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~ms_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

ms_status ms_graph_create(ms_batch* b, const float* dev_targets, int32_t steps_per_launch, int32_t n_launches,
                          ms_graph** out) {
    if (!b || !out) return fail(MS_E_INVALID_ARG, "null batch or output handle");
    *out = nullptr;
    if (steps_per_launch < 1 || n_launches < 1 || n_launches > 100000)
        return fail(MS_E_INVALID_ARG, "steps_per_launch must be >= 1 and n_launches in [1, 100000] (got %d, %d)",
                    steps_per_launch, n_launches);
    HIP_OK(hipSetDevice(b->device));
    if (ms_status st = ensure_side_streams(b); st != MS_OK) return st;
    hipStream_t cap = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    std::unique_ptr<ms_graph> g(new ms_graph());
    g->b = b;
    g->plan_gen = b->plan_gen;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    ms_status st = e == hipSuccess ? MS_OK : fail(MS_E_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    if (st == MS_OK) {
        for (int k = 0; k < n_launches && st == MS_OK; ++k) st = ms_step(b, dev_targets, steps_per_launch, cap);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap, &graph);   // always end the capture, also after a failed step
        g->graph = graph;
        if (st == MS_OK && e != hipSuccess) st = fail(MS_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    if (st == MS_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = fail(MS_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cap);
    if (st != MS_OK) return st;
    *out = g.release();
    return MS_OK;
}

ms_status ms_graph_launch(ms_graph* g, void* hip_stream) {
    if (!g || !g->exec) return fail(MS_E_INVALID_ARG, "null graph");
    if (g->plan_gen != g->b->plan_gen)
        return fail(MS_E_STATE, "the batch was re-planned (ms_tune_batch) after this graph was captured: "
                                "destroy the graph and capture it again");
    HIP_OK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(hip_stream)));
    return MS_OK;
}

ms_status ms_graph_destroy(ms_graph* g) {
    delete g;
    return MS_OK;
}

static size_t many_bytes(ms_batch* const* batches, int32_t n) {
    size_t tiles = 0, tenv = 0;
    for (int i = 0; i < n; ++i) { tiles += batches[i]->plan.tiles.size(); tenv += batches[i]->plan.tenv.size(); }
    return align_up(size_t(n) * sizeof(BatchDev)) + align_up(tiles * sizeof(Tile)) + align_up(tenv * sizeof(TileEnv)) +
           align_up(tiles * sizeof(Bin));
}

ms_status ms_query_step_many_bytes(ms_batch* const* batches, int32_t n_batches, size_t* bytes) {
    if (!batches || n_batches <= 0 || !bytes) return fail(MS_E_INVALID_ARG, "bad arguments");
    for (int i = 0; i < n_batches; ++i)
        if (!batches[i]) return fail(MS_E_INVALID_ARG, "null batch %d", i);
    *bytes = many_bytes(batches, n_batches);
    return MS_OK;
}

namespace {
// Pinned host staging for the combined work list, reused once the previous upload completed,
// and the side streams of the LDS-class fork / join (one set per host thread and device).
// The thread that loaded the library (the process's main thread in practice): its staging is
// left to process exit, when the runtime may already be going away.
const std::thread::id g_load_thread = std::this_thread::get_id();
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    int device = -1;
    bool pending = false;
    hipStream_t side[MAX_CLASSES] = {};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[MAX_CLASSES] = {};
    // Wait for this thread's last upload and launches, then free its pinned buffer, events and
    // side streams (a server worker thread's staging, when the worker exits).
    void release() {
        if (ev) { (void)hipEventSynchronize(ev); (void)hipEventDestroy(ev); ev = nullptr; }
        for (int k = 0; k < MAX_CLASSES; ++k) {
            if (side[k]) { (void)hipStreamSynchronize(side[k]); (void)hipStreamDestroy(side[k]); side[k] = nullptr; }
            if (ev_join[k]) { (void)hipEventDestroy(ev_join[k]); ev_join[k] = nullptr; }
        }
        if (ev_fork) { (void)hipEventDestroy(ev_fork); ev_fork = nullptr; }
        if (host) { (void)hipHostFree(host); host = nullptr; }
        cap = 0;
        pending = false;
        device = -1;
    }
    ~Staging() {
        if (std::this_thread::get_id() != g_load_thread) release();
    }
};
thread_local Staging g_stage;

struct ManyTile {
    int lds_words, batch, tile;
    bool one;
};
}  // namespace

ms_status ms_step_many(ms_batch* const* batches, const float* const* dev_targets, int32_t n_batches, int32_t n_steps,
                       void* dev_scratch, size_t scratch_bytes, void* hip_stream) {
    if (!batches || n_batches <= 0) return fail(MS_E_INVALID_ARG, "bad batch list");
    if (n_steps < 1) return fail(MS_E_INVALID_ARG, "n_steps must be >= 1");
    for (int i = 0; i < n_batches; ++i)
        if (!batches[i]) return fail(MS_E_INVALID_ARG, "null batch %d", i);
    const size_t need = many_bytes(batches, n_batches);
    if (!dev_scratch || scratch_bytes < need)
        return fail(MS_E_NO_WORKSPACE, "scratch of %zu bytes, %zu needed", scratch_bytes, need);
    if (reinterpret_cast<uintptr_t>(dev_scratch) % ALIGN) return fail(MS_E_INVALID_ARG, "scratch must be 256-byte aligned");
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    for (int i = 0; i < n_batches; ++i)
        if (batches[i]->device != dev) return fail(MS_E_INVALID_ARG, "batch %d lives on device %d, not %d", i, batches[i]->device, dev);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int opt = 0;
    for (int i = 0; i < n_batches; ++i) opt |= batch_opt(batches[i]);
    Staging& st = g_stage;
    if (st.device != dev) {
        st.release();
        st.device = dev;
        HIP_OK(hipEventCreateWithFlags(&st.ev, hipEventDisableTiming));
    }
    if (st.pending) { HIP_OK(hipEventSynchronize(st.ev)); st.pending = false; }
    if (st.cap < need) {
        if (st.host) HIP_OK(hipHostFree(st.host));
        st.host = nullptr;
        st.cap = 0;
        HIP_OK(hipHostMalloc(&st.host, need, hipHostMallocDefault));
        st.cap = need;
    }
    char* h = static_cast<char*>(st.host);
    BatchDev* tb = reinterpret_cast<BatchDev*>(h);
    Tile* tt = reinterpret_cast<Tile*>(h + align_up(size_t(n_batches) * sizeof(BatchDev)));
    size_t n_tiles = 0;
    for (int i = 0; i < n_batches; ++i) n_tiles += batches[i]->plan.tiles.size();
    TileEnv* te = reinterpret_cast<TileEnv*>(reinterpret_cast<char*>(tt) + align_up(n_tiles * sizeof(Tile)));
    // env slots batch by batch; tiles of all batches merged and ordered by LDS need (largest
    // first), then cut into LDS classes by the rule of the single-batch plan
    std::vector<int> tenv_base(n_batches + 1, 0);
    std::vector<ManyTile> order;
    order.reserve(n_tiles);
    for (int i = 0; i < n_batches; ++i) {
        ms_batch* b = batches[i];
        tb[i] = b->hbd;
        tenv_base[i + 1] = tenv_base[i] + int(b->plan.tenv.size());
        for (size_t k = 0; k < b->plan.tenv.size(); ++k) {
            TileEnv f = b->plan.tenv[k];
            f.batch = i;
            te[tenv_base[i] + k] = f;
        }
        for (size_t t = 0; t < b->plan.tiles.size(); ++t) {
            const Tile& u = b->plan.tiles[t];
            order.push_back(ManyTile{u.lds_words, i, int(t), u.lanes == WAVE && u.count == 1});
        }
        if (dev_targets && dev_targets[i] && b->J > 0)
            HIP_OK(hipMemcpyAsync(const_cast<float*>(b->hbd.targets), dev_targets[i], size_t(b->J) * 4,
                                  hipMemcpyDeviceToDevice, s));
    }
    std::stable_sort(order.begin(), order.end(), [](const ManyTile& a, const ManyTile& b) { return a.lds_words > b.lds_words; });
    std::vector<LdsClass> cls;
    for (size_t k = 0; k < order.size(); ++k) {
        Tile u = batches[order[k].batch]->plan.tiles[order[k].tile];
        u.first += tenv_base[order[k].batch];
        tt[k] = u;
    }
    cut_classes(int(order.size()), [&](int k) -> Tile& { return tt[k]; }, true, cls);
    // several LDS sizes: one launch of bins (as for a single batch)
    Bin* hb = reinterpret_cast<Bin*>(reinterpret_cast<char*>(te) + align_up(size_t(tenv_base[n_batches]) * sizeof(TileEnv)));
    std::vector<Bin> bins;
    std::vector<int> used;
    int bin_words = 0;
    if (cls.size() > 1) {
        bin_words = pack_bins(int(order.size()), [&](int k) -> const Tile& { return tt[k]; }, bins, used);
        std::copy(bins.begin(), bins.end(), hb);
    }
    HIP_OK(hipMemcpyAsync(dev_scratch, st.host, need, hipMemcpyHostToDevice, s));
    HIP_OK(hipEventRecord(st.ev, s));
    st.pending = true;
    char* d = static_cast<char*>(dev_scratch);
    const BatchDev* dtb = reinterpret_cast<const BatchDev*>(d);
    const Tile* dtt = reinterpret_cast<const Tile*>(d + (reinterpret_cast<char*>(tt) - h));
    const TileEnv* dte = reinterpret_cast<const TileEnv*>(d + (reinterpret_cast<char*>(te) - h));
    if (!bins.empty()) {
        const Bin* dbins = reinterpret_cast<const Bin*>(d + (reinterpret_cast<char*>(hb) - h));
        const int nb = int(bins.size());
        hipLaunchKernelGGL(bins_kernel(opt), dim3(nb), dim3(WAVE * BIN_WAVES), size_t(bin_words) * 4, s, dtb, dtt, dbins,
                           nb, dte, int(n_steps));
        HIP_OK(hipGetLastError());
        return MS_OK;
    }
    if (cls.size() > 1 && !st.ev_fork) {
        HIP_OK(hipEventCreateWithFlags(&st.ev_fork, hipEventDisableTiming));
        for (int k = 1; k < MAX_CLASSES; ++k) {
            HIP_OK(hipStreamCreateWithFlags(&st.side[k], hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&st.ev_join[k], hipEventDisableTiming));
        }
    }
    if (cls.size() > 1) HIP_OK(hipEventRecord(st.ev_fork, s));
    for (size_t k = 0; k < cls.size(); ++k) {
        hipStream_t sk = k == 0 ? s : st.side[k];
        if (k > 0) HIP_OK(hipStreamWaitEvent(sk, st.ev_fork, 0));
        if (ms_status r = launch_class(cls[k], dtb, dtt, dte, int(n_steps), 0, sk, opt); r != MS_OK) return r;
        if (k > 0) {
            HIP_OK(hipEventRecord(st.ev_join[k], sk));
            HIP_OK(hipStreamWaitEvent(s, st.ev_join[k], 0));
        }
    }
    return MS_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------- fused step, no allocation
// Work-list scratch of ms_step_many_noalloc: a file-scope device array, one copy per GPU that the
// library runs on, held until the process ends.  Host code never uses its name as an address:
// each device's copy is found once with hipGetSymbolAddress and that pointer is what the
// upload and the kernels receive.
static __device__ __align__(256) unsigned char scratch[MS_STEP_MANY_NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr int NOALLOC_MAX_BATCHES = 4096;
constexpr size_t NOALLOC_MAX_TILES = MS_STEP_MANY_NOALLOC_BYTES / sizeof(Tile);
// Host side of the entry point, all static: the per-device scratch addresses, the host image of
// the work list (uploaded from pageable memory: the copy call returns once the runtime has
// taken the bytes, so the image may be rebuilt by the next call) and the planner's working
// arrays.  One mutex serialises the host part of concurrent calls.
std::mutex g_noalloc_mu;
void* g_noalloc_dev[NOALLOC_MAX_DEVICES] = {};
alignas(256) unsigned char g_noalloc_host[MS_STEP_MANY_NOALLOC_BYTES];
int g_noalloc_used[NOALLOC_MAX_TILES];
int g_noalloc_head[NOALLOC_MAX_BATCHES];
int g_noalloc_tenv_base[NOALLOC_MAX_BATCHES + 1];
LdsClass g_noalloc_cls[MAX_CLASSES];
}  // namespace

extern "C" {

ms_status ms_step_many_noalloc(ms_batch* const* batches, const float* const* dev_targets, int32_t n_batches,
                               int32_t n_steps, void* hip_stream) {
    if (!batches || n_batches <= 0) return fail(MS_E_INVALID_ARG, "bad batch list");
    if (n_steps < 1) return fail(MS_E_INVALID_ARG, "n_steps must be >= 1");
    if (n_batches > NOALLOC_MAX_BATCHES)
        return fail(MS_E_CAPACITY, "%d batches, at most %d in one call", n_batches, NOALLOC_MAX_BATCHES);
    for (int i = 0; i < n_batches; ++i)
        if (!batches[i]) return fail(MS_E_INVALID_ARG, "null batch %d", i);
    const size_t need = many_bytes(batches, n_batches);
    if (need > size_t(MS_STEP_MANY_NOALLOC_BYTES))
        return fail(MS_E_CAPACITY, "the fused work list needs %zu bytes, more than the %u-byte static scratch "
                    "(use ms_step_many with caller scratch)", need, unsigned(MS_STEP_MANY_NOALLOC_BYTES));
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(MS_E_DEVICE, "device %d beyond the library's table", dev);
    for (int i = 0; i < n_batches; ++i)
        if (batches[i]->device != dev) return fail(MS_E_INVALID_ARG, "batch %d lives on device %d, not %d", i, batches[i]->device, dev);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int opt = 0;
    for (int i = 0; i < n_batches; ++i) opt |= batch_opt(batches[i]);

    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_dev[dev]) {
        // first call on this device (current): its own copy of the array
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MS_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
        g_noalloc_dev[dev] = p;
    }
    char* d = static_cast<char*>(g_noalloc_dev[dev]);
    char* h = reinterpret_cast<char*>(g_noalloc_host);

    // host image: batch table, merged tiles, env slots, bins (the layout of ms_step_many)
    size_t n_tiles = 0;
    for (int i = 0; i < n_batches; ++i) n_tiles += batches[i]->plan.tiles.size();
    BatchDev* tb = reinterpret_cast<BatchDev*>(h);
    Tile* tt = reinterpret_cast<Tile*>(h + align_up(size_t(n_batches) * sizeof(BatchDev)));
    TileEnv* te = reinterpret_cast<TileEnv*>(reinterpret_cast<char*>(tt) + align_up(n_tiles * sizeof(Tile)));
    int* tenv_base = g_noalloc_tenv_base;
    tenv_base[0] = 0;
    for (int i = 0; i < n_batches; ++i) {
        ms_batch* b = batches[i];
        tb[i] = b->hbd;
        tenv_base[i + 1] = tenv_base[i] + int(b->plan.tenv.size());
        for (size_t k = 0; k < b->plan.tenv.size(); ++k) {
            TileEnv f = b->plan.tenv[k];
            f.batch = i;
            te[tenv_base[i] + k] = f;
        }
        g_noalloc_head[i] = 0;
        if (dev_targets && dev_targets[i] && b->J > 0)
            HIP_OK(hipMemcpyAsync(const_cast<float*>(b->hbd.targets), dev_targets[i], size_t(b->J) * 4,
                                  hipMemcpyDeviceToDevice, s));
    }
    // merge the batches' tile lists (each ordered by LDS need, largest first) into one list of
    // the same order, earlier batches first among equals
    for (size_t k = 0; k < n_tiles; ++k) {
        int best = -1, best_words = -1;
        for (int i = 0; i < n_batches; ++i) {
            const std::vector<Tile>& T = batches[i]->plan.tiles;
            if (g_noalloc_head[i] < int(T.size()) && T[g_noalloc_head[i]].lds_words > best_words) {
                best = i;
                best_words = T[g_noalloc_head[i]].lds_words;
            }
        }
        Tile u = batches[best]->plan.tiles[g_noalloc_head[best]++];
        u.first += tenv_base[best];
        tt[k] = u;
    }
    FixedVec<LdsClass> cls(g_noalloc_cls, MAX_CLASSES);
    cut_classes(int(n_tiles), [&](int k) -> Tile& { return tt[k]; }, true, cls);
    Bin* hb = reinterpret_cast<Bin*>(reinterpret_cast<char*>(te) + align_up(size_t(tenv_base[n_batches]) * sizeof(TileEnv)));
    FixedVec<Bin> bins(hb, n_tiles);
    FixedVec<int> used(g_noalloc_used, n_tiles);
    int bin_words = 0;
    if (cls.size() > 1) bin_words = pack_bins(int(n_tiles), [&](int k) -> const Tile& { return tt[k]; }, bins, used);
    HIP_OK(hipMemcpyAsync(d, h, need, hipMemcpyHostToDevice, s));
    const BatchDev* dtb = reinterpret_cast<const BatchDev*>(d);
    const Tile* dtt = reinterpret_cast<const Tile*>(d + (reinterpret_cast<char*>(tt) - h));
    const TileEnv* dte = reinterpret_cast<const TileEnv*>(d + (reinterpret_cast<char*>(te) - h));
    if (cls.size() > 1) {
        const Bin* dbins = reinterpret_cast<const Bin*>(d + (reinterpret_cast<char*>(hb) - h));
        const int nb = int(bins.size());
        hipLaunchKernelGGL(bins_kernel(opt), dim3(nb), dim3(WAVE * BIN_WAVES), size_t(bin_words) * 4, s, dtb, dtt, dbins,
                           nb, dte, int(n_steps));
        HIP_OK(hipGetLastError());
        return MS_OK;
    }
    return launch_class(cls[0], dtb, dtt, dte, int(n_steps), 0, s, opt);
}

}  // extern "C"

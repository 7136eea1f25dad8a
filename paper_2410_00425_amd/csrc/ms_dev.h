// ms_dev.h — library-internal types shared by the host runtime and the step kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msdev {

constexpr int WAVE = 64;
constexpr int MAX_BODIES = 64;
constexpr int MAX_JOINTS = 64;
constexpr int PLANE = 0xFFFF;
constexpr int N_COLOURS = 64;  // colours 0..63 are parallel; colour 64 is the serial overflow

// Body parameter record in HBM: three float4 per body, component-plane major ([3][B]):
//   p0 = {shape | flags << 8 (int bits), inverse mass, friction, restitution}
//   p1 = {dim0, dim1, dim2, 0}
//   p2 = {principal inverse inertia x, y, z, 0}
// Joint record in HBM: JREC floats per joint: parent, child (int bits), anchor A (3), frame
// rotation A (4), anchor B (3), frame rotation B (4), kp, kd, type | limited << 8 (int bits),
// lower, upper, 0.
constexpr int JREC = 22;
enum { JOINT_REVOLUTE = 0, JOINT_PRISMATIC = 1 };

// One batch as the kernels see it (device memory, read by every tile of the batch).
struct BatchDev {
    float* pos;     // [3][B]
    float* quat;    // [4][B]
    float* vel;     // [3][B]
    float* angvel;  // [3][B]
    int* status;    // [E]
    const float4* bpar;   // [3][B]
    const int* body_off;  // [E + 1]
    const int* joint_off; // [E + 1]
    const float* jrec;    // [J][JREC]
    const float* targets; // [J]
    int B, E, J, pad0;
    // step model parameters
    float dt, gx, gy, gz;
    int S, K, V, JI;       // substeps, iterations per substep, velocity iterations, joint passes
    float plane_z, plane_mu, plane_e, delta;
    int plane, pad1, pad2, pad3;
    float beta, max_depen, beta_j, bounce;
    float lin_damp, ang_damp, pad4, pad5;
    // debug export of the last step of a launch (null when off)
    int* dbg_pairs;        // [sum P_e][4]: a, b, kept points, decision
    const int* dbg_pair_off;
    float* dbg_pts;        // [sum cap_e][8]: p (3), n (3), s0, lambda_n
    const int* dbg_pt_off;
    float* dbg_man;        // [sum mcap_e][8]: pair index, colour, lt1, lt2, ltw, mu, rt, count
    const int* dbg_man_off;
    int* dbg_counts;       // [E][4]: candidates, points, manifolds, colours
    // work counters, accumulated over launches in 64 bits: [E][NSTAT] (see STAT_*)
    long long* stats;
    // net contact force on every body over the last step of a launch, [3][B] (null: not computed)
    float* forces;
    // count of env ids outside [0, E) met by the reset kernels
    int* bad_ids;
    // cross-step warm start: the contact cache of the last step (null when off).  Per env: header
    // {manifolds, points}; manifold records {pair key, first | count << 16 (int bits), tangential
    // impulse vector (3), twist impulse} at cache_man_off[e]; point records {position in body B's
    // frame at the step start (3), normal impulse} at cache_pt_off[e]
    int* cache_hdr;
    float* cache_man;
    const int* cache_man_off;
    float* cache_pt;
    const int* cache_pt_off;
    float warm_radius;
    int pad6;
    // per-phase wave-cycles, [16], summed over the launches (only in the per-phase clock build)
    unsigned long long* phase_clock;
    // compound table (null when the batch has none): COMP_WORDS floats per compound, {parts (int
    // bits), 0, 0, 0} then per part {shape (int bits), dims (3)}, {position (3), qw},
    // {qx, qy, qz, 0}; a compound body's dim0 holds its table index
    const float* comp;
    int n_comp, pad7;
};
constexpr int CM_WORDS = 6, CP_WORDS = 4;
constexpr int MAX_PARTS = 4, COMP_WORDS = 4 + 12 * MAX_PARTS;
constexpr int SHAPE_COMPOUND = 3;

// Work counters per env: steps, candidate pairs per shape kind (3 * min + max shape for body
// pairs, 9 + shape for plane pairs), contact points, manifolds, colours.
enum { STAT_STEPS = 0, STAT_KIND0 = 1, STAT_POINTS = 13, STAT_MANIFOLDS = 14, STAT_COLOURS = 15, NSTAT = 16 };

// One env slot of a tile (host-computed).
struct TileEnv {
    int batch;    // index into the launch's batch table
    int env;      // env id within the batch
    int lds_off;  // word offset of the env's LDS region within the workgroup's LDS
    int n;        // bodies
    int nj;       // joints
    int cap;      // contact point capacity
    int mcap;     // manifold capacity
    int pad;
};

// A tile: `count` envs (consecutive TileEnv records from `first`), `lanes` lanes per env.
struct Tile {
    int first;
    int count;
    int lanes;
    int lds_words;
};

// A bin: up to BIN_WAVES tiles run by the wavefronts of one workgroup, tile k at word offset
// off[k] of the workgroup's LDS (the single-launch form of a batch with tiles of several sizes).
constexpr int BIN_WAVES = 4;
struct Bin {
    int count;
    int tile[BIN_WAVES];
    int off[BIN_WAVES];
};

// Word offsets of one env's arrays: component-major planes of length n, except the per-body
// solver records and the contact, manifold and joint rows, which are records.
enum { B_V = 0, B_W = 3, B_IM = 6, B_IW = 7, BODY_WORDS = 13 };
enum { P_DX = 0, P_DQ = 3, P_X0 = 7, P_QC = 10, P_Q0 = 14, POSE_WORDS = 18 };
struct Lay {
    int n, nj, cap, mcap, P;
    // bodies
    int POSE, BODY, V0, W0, IB, AABB, SH, DIM, MU, EE, CM, JM;
    int JNT, JINV, CAND, PT, MAN, BCOL, ORDER, SCHED, JSCHED, CSTART, SCAL;
    int total;  // words, a multiple of 4
};
__host__ __device__ inline Lay make_lay(int n, int nj, int cap, int mcap) {
    Lay L;
    L.n = n; L.nj = nj; L.cap = cap; L.mcap = mcap; L.P = n * (n + 1) / 2;
    int o = 0;
    // pose record of a body, POSE_WORDS per body: substep offsets dx (3), dq (4), step-start
    // position (3), current orientation (4), step-start orientation (4)
    L.POSE = o; o += POSE_WORDS * n;
    // solver record of a body, BODY_WORDS per body: v (3), w (3), inverse mass, world inverse
    // inertia frozen for the step (xx, yy, zz, xy, xz, yz)
    L.BODY = o; o += BODY_WORDS * n;
    L.V0 = o; o += 3 * n;
    L.W0 = o; o += 3 * n;
    L.IB = o; o += 3 * n;  // principal inverse inertia (body frame)
    L.AABB = o; o += 6 * n;
    L.SH = o; o += n;
    L.DIM = o; o += 3 * n;
    L.MU = o; o += n;
    L.EE = o; o += n;
    L.CM = o; o += 2 * n;  // colour masks (u64)
    L.JM = o; o += 2 * n;  // jointed-partner masks (u64)
    // 55 n words so far
    L.JNT = o; o += 31 * nj;    // joint records (J_WORDS)
    L.JINV = o; o += 40 * nj;   // per-joint quantities fixed within a substep (JI_WORDS)

    // candidate pairs (u16) during S2-S4; afterwards the per-body block lists (offsets [n + 1],
    // entries u16 [2 (nj + mcap)])
    L.CAND = o; o += (L.P + 1) / 2 > n + 1 + nj + mcap ? (L.P + 1) / 2 : n + 1 + nj + mcap;
    L.PT = o; o += 14 * cap;
    L.MAN = o; o += 23 * mcap;
    L.BCOL = o; o += (nj + mcap + 1) / 2;
    L.ORDER = o; o += (nj + mcap + 1) / 2;
    L.SCHED = o; o += nj + mcap + 66;
    L.JSCHED = o; o += nj > 0 ? nj + mcap + 66 : 66;  // without joints: cursors of the serial colouring only
    L.CSTART = o; o += 68;
    L.SCAL = o; o += 32;  // 16 scalars + 16 work counters
    L.total = (o + 3) & ~3;
    return L;
}
// LDS words needed by one env.
inline int env_lds_words(int n, int nj, int cap, int mcap) { return make_lay(n, nj, cap, mcap).total; }

// Pair index k in canonical order -> (a, b) with a < b <= n (b = n is the plane).
__host__ __device__ inline void pair_of(int k, int n, int& a, int& b) {
    // row a starts at a (2n - a + 1) / 2
    float fn = float(2 * n + 1);
    int aa = int((fn - sqrtf(fn * fn - 8.0f * float(k))) * 0.5f);
    aa = (aa < 0 ? 0 : (aa > n - 1 ? n - 1 : aa));
    while (aa > 0 && aa * (2 * n - aa + 1) / 2 > k) --aa;
    while (aa + 1 < n && (aa + 1) * (2 * n - aa) / 2 <= k) ++aa;
    a = aa;
    b = a + 1 + (k - a * (2 * n - a + 1) / 2);
}


}  // namespace msdev

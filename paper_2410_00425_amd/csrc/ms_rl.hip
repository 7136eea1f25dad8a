// ms_rl.hip — device kernels of the learning-loop calls (all on the batch's stream, no host
// synchronisation): seeded randomised partial resets, the target-delta joint controller, joint
// positions and drive targets.  The per-body contact forces are accumulated by the step kernel.
//
// Randomised reset (the paper's partial resets with per-env seeded randomisation of the
// initial robot configuration and of object placement; App. C PPO partial resets, Sec. III-G
// per-env seeding):  from the batch's initial state, every free dynamic body (the child of no
// joint) moves by xy_half (2u - 1) in x and in y and turns about the world z axis through its
// centre by yaw_half (2u - 1); every joint in index order takes the position
// q0 = q_init + joint_sigma N, N a standard normal deviate, and poses its child from its parent
// (forward kinematics); velocities are zero and the status is cleared; optionally the drive
// target becomes q0.  Random numbers: Philox4x32-10 (Salmon et al., SC'11) under the 64-bit key
// `seed`, counter (env, reset count, purpose, index): body i draws block (1, i), joint j the
// blocks (0, 3j .. 3j + 2) whose 12 uniforms sum to an Irwin-Hall deviate minus 6.  sin and cos
// of the half angles come from their Taylor series (correctly rounded operations only, so the
// result is reproducible bit for bit on any IEEE machine).

// Philox4x32-10: ten rounds of the multiply-xor bijection, the key bumped by the Weyl constants
// between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}
// A uniform in [0, 1) from the top 24 bits of a 32-bit draw (exact in float).
__device__ __forceinline__ float unit24(uint32_t x) { return float(x >> 8) * 5.9604644775390625e-08f; }

// sin / cos by Taylor series in x^2 (Horner), to x^17 / x^18: truncation below 1e-11 on
// [-pi/2 - 0.2, pi/2 + 0.2].
__device__ __forceinline__ float sin_series(float x) {
    const float x2 = x * x;
    float p = 1.0f / 355687428096000.0f;
    p = -1.0f / 1307674368000.0f + x2 * p;
    p = 1.0f / 6227020800.0f + x2 * p;
    p = -1.0f / 39916800.0f + x2 * p;
    p = 1.0f / 362880.0f + x2 * p;
    p = -1.0f / 5040.0f + x2 * p;
    p = 1.0f / 120.0f + x2 * p;
    p = -1.0f / 6.0f + x2 * p;
    p = 1.0f + x2 * p;
    return x * p;
}
__device__ __forceinline__ float cos_series(float x) {
    const float x2 = x * x;
    float p = -1.0f / 6402373705728000.0f;
    p = 1.0f / 20922789888000.0f + x2 * p;
    p = -1.0f / 87178291200.0f + x2 * p;
    p = 1.0f / 479001600.0f + x2 * p;
    p = -1.0f / 3628800.0f + x2 * p;
    p = 1.0f / 40320.0f + x2 * p;
    p = -1.0f / 720.0f + x2 * p;
    p = 1.0f / 24.0f + x2 * p;
    p = -1.0f / 2.0f + x2 * p;
    return 1.0f + x2 * p;
}

struct ResetNoiseDev {
    float joint_sigma, xy_half, yaw_half;
    int targets_follow;
};

__device__ __forceinline__ V3 ldg3(const float* a, int B, int i) { return v3(a[i], a[B + i], a[2 * B + i]); }
__device__ __forceinline__ Qt ldg4(const float* a, int B, int i) { return Qt{a[i], a[B + i], a[2 * B + i], a[3 * B + i]}; }
__device__ __forceinline__ void stg3(float* a, int B, int i, V3 v) { a[i] = v.x; a[B + i] = v.y; a[2 * B + i] = v.z; }
__device__ __forceinline__ void stg4(float* a, int B, int i, Qt q) { a[i] = q.w; a[B + i] = q.x; a[2 * B + i] = q.y; a[3 * B + i] = q.z; }

// Position of joint record J (HBM layout, see JREC) from poses given as SoA planes: the twist
// 2 atan2(q_rel.z, q_rel.w) (q_rel.w >= 0) of the child's joint frame relative to the parent's
// (revolute), or the anchors' separation along the slide axis (prismatic); the same operations
// as the step's joint frame.  b0: the env's first body in the planes.
__device__ __forceinline__ float joint_position_soa(const float* J, const float* pos, const float* quat, int B, int b0) {
    const int pa = __float_as_int(J[0]), ch = __float_as_int(J[1]);
    const Qt qa = pa >= 0 ? ldg4(quat, B, b0 + pa) : Qt{1.0f, 0.0f, 0.0f, 0.0f};
    const Qt qb = ldg4(quat, B, b0 + ch);
    const Qt QA = Qt{J[5], J[6], J[7], J[8]}, QB = Qt{J[12], J[13], J[14], J[15]};
    const bool prism = (__float_as_int(J[18]) & 0xFF) == JOINT_PRISMATIC;
    if (prism) {
        const V3 xa = pa >= 0 ? ldg3(pos, B, b0 + pa) : v3(0, 0, 0);
        const V3 rA = mulv(rotm(qa), v3(J[2], J[3], J[4]));
        const V3 rB = mulv(rotm(qb), v3(J[9], J[10], J[11]));
        const V3 zA = colm(rotm(qmul(qa, QA)), 2);
        const V3 d = (ldg3(pos, B, b0 + ch) + rB) - (xa + rA);
        return dot3(zA, d);
    }
    const Qt qaf = qmul(qa, QA), qbf = qmul(qb, QB);
    Qt rel = qmul(Qt{qaf.w, -qaf.x, -qaf.y, -qaf.z}, qbf);
    if (rel.w < 0.0f) rel = Qt{-rel.w, -rel.x, -rel.y, -rel.z};
    return 2.0f * atan2_w(rel.z, rel.w);
}

// One thread per listed env (serial over its bodies, then its joints in index order).  Ids
// outside [0, E) are skipped and counted in *bad_ids.  ipos / iquat: the initial state planes.
extern "C" __global__ void __launch_bounds__(64) ms_reset_random_kernel(BatchDev bd, const int* __restrict__ env_ids,
                                                                      int n_ids, const float* __restrict__ ipos,
                                                                      const float* __restrict__ iquat, ResetNoiseDev nz,
                                                                      uint32_t key0, uint32_t key1, uint32_t count,
                                                                      int* __restrict__ bad_ids) {
    const int k = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (k >= n_ids) return;
    const int e = env_ids[k];
    if (e < 0 || e >= bd.E) { atomicAdd(bad_ids, 1); return; }
    const int B = bd.B;
    const int b0 = bd.body_off[e], n = bd.body_off[e + 1] - b0;
    const int j0 = bd.joint_off[e], nj = bd.joint_off[e + 1] - j0;
    uint64_t child = 0;
    for (int j = 0; j < nj; ++j) child |= uint64_t(1) << __float_as_int(bd.jrec[size_t(j0 + j) * JREC + 1]);
    for (int i = 0; i < n; ++i) {
        const int gi = b0 + i;
        V3 x = ldg3(ipos, B, gi);
        Qt q = ldg4(iquat, B, gi);
        const bool dyn = !((__float_as_int(bd.bpar[gi].x) >> 8) & 1);
        if (dyn && !((child >> i) & 1)) {
            uint32_t u[4];
            philox4x32_10(uint32_t(e), count, 1u, uint32_t(i), key0, key1, u);
            x.x = x.x + nz.xy_half * (2.0f * unit24(u[0]) - 1.0f);
            x.y = x.y + nz.xy_half * (2.0f * unit24(u[1]) - 1.0f);
            const float half = 0.5f * (nz.yaw_half * (2.0f * unit24(u[2]) - 1.0f));
            q = qnorm(qmul(Qt{cos_series(half), 0.0f, 0.0f, sin_series(half)}, q));
        }
        stg3(bd.pos, B, gi, x);
        stg4(bd.quat, B, gi, q);
        stg3(bd.vel, B, gi, v3(0, 0, 0));
        stg3(bd.angvel, B, gi, v3(0, 0, 0));
        if (bd.forces) stg3(bd.forces, B, gi, v3(0, 0, 0));
    }
    for (int j = 0; j < nj; ++j) {
        const float* J = bd.jrec + size_t(j0 + j) * JREC;
        // the joint's position in the initial state, plus the drawn offset
        const float q_init = joint_position_soa(J, ipos, iquat, B, b0);
        float sum = 0.0f;
        for (uint32_t blk = 0; blk < 3; ++blk) {
            uint32_t u[4];
            philox4x32_10(uint32_t(e), count, 0u, uint32_t(3 * j) + blk, key0, key1, u);
            for (int r = 0; r < 4; ++r) sum = sum + unit24(u[r]);
        }
        const float q0 = q_init + nz.joint_sigma * (sum - 6.0f);
        // forward kinematics from the (already placed) parent
        const int pa = __float_as_int(J[0]), ch = __float_as_int(J[1]);
        const bool prism = (__float_as_int(J[18]) & 0xFF) == JOINT_PRISMATIC;
        const Qt qp = pa >= 0 ? ldg4(bd.quat, B, b0 + pa) : Qt{1.0f, 0.0f, 0.0f, 0.0f};
        const V3 xp = pa >= 0 ? ldg3(bd.pos, B, b0 + pa) : v3(0, 0, 0);
        const Qt qpf = qmul(qp, Qt{J[5], J[6], J[7], J[8]});
        const Qt rot = prism ? Qt{1.0f, 0.0f, 0.0f, 0.0f}
                             : Qt{cos_series(0.5f * q0), 0.0f, 0.0f, sin_series(0.5f * q0)};
        const Qt qc = qnorm(qmul(qmul(qpf, rot), Qt{J[12], -J[13], -J[14], -J[15]}));
        V3 anchor = xp + mulv(rotm(qp), v3(J[2], J[3], J[4]));
        if (prism) anchor = anchor + q0 * colm(rotm(qpf), 2);
        const V3 xc = anchor - mulv(rotm(qc), v3(J[9], J[10], J[11]));
        stg3(bd.pos, B, b0 + ch, xc);
        stg4(bd.quat, B, b0 + ch, qc);
        if (nz.targets_follow) const_cast<float*>(bd.targets)[j0 + j] = q0;
    }
    bd.status[e] = 0;
    if (bd.cache_hdr) { bd.cache_hdr[2 * e] = 0; bd.cache_hdr[2 * e + 1] = 0; }
}

// Target-delta joint position controller: target += clip(a, -1, 1) (high - low) / 2 per joint,
// float32 (the paper's delta joint-position action space; low / high per joint or scalars).
extern "C" __global__ void __launch_bounds__(256) ms_apply_actions_kernel(float* __restrict__ targets,
                                                                        const float* __restrict__ actions,
                                                                        const float* __restrict__ low,
                                                                        const float* __restrict__ high, float lo,
                                                                        float hi, int J) {
    const int j = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (j >= J) return;
    const float a = actions[j];
    const float c = a < -1.0f ? -1.0f : (a > 1.0f ? 1.0f : a);
    const float l = low ? low[j] : lo, u = high ? high[j] : hi;
    targets[j] = targets[j] + c * (0.5f * (u - l));
}

// Joint positions of the current state, float32 [J]: one thread per env.
extern "C" __global__ void __launch_bounds__(64) ms_joint_positions_kernel(BatchDev bd, float* __restrict__ out) {
    const int e = int(blockIdx.x) * 64 + int(threadIdx.x);
    if (e >= bd.E) return;
    const int b0 = bd.body_off[e], j0 = bd.joint_off[e], j1 = bd.joint_off[e + 1];
    for (int j = j0; j < j1; ++j) out[j] = joint_position_soa(bd.jrec + size_t(j) * JREC, bd.pos, bd.quat, bd.B, b0);
}

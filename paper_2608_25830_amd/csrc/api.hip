// api.hip -- the C ABI of include/gtmp.h: host-side validation, translation of
// the public structs into kernel arguments, and dispatch to the launchers.
// No C++ exception crosses the boundary; every failure returns a status and
// records a thread-local message.
#include <cmath>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "gtmp_launch.hpp"
#include "surrogate.hpp"

namespace {

thread_local char g_err[512] = "";

gtmp_status fail(gtmp_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

gtmp_status hip_status(hipError_t e, const char *where) {
    if (e == hipSuccess) return GTMP_OK;
    return fail(GTMP_EHIP, "%s: %s", where, hipGetErrorString(e));
}

gtmp_status check_problem(const gtmp_problem *p) {
    if (!p) return fail(GTMP_EINVAL, "problem is NULL");
    if (p->d < 1 || p->d > GTMP_MAX_DOF) return fail(GTMP_EINVAL, "d=%d outside 1..%d", p->d, GTMP_MAX_DOF);
    if (p->M < 1) return fail(GTMP_EINVAL, "M=%d < 1", p->M);
    if (p->N < 1) return fail(GTMP_EINVAL, "N=%d < 1", p->N);
    if (p->G < 1) return fail(GTMP_EINVAL, "G=%d < 1", p->G);
    if (p->H < 2 || p->H > GTMP_MAX_H) return fail(GTMP_EINVAL, "H=%d outside 2..%d", p->H, GTMP_MAX_H);
    for (int j = 0; j < p->d; ++j)
        if (!(isfinite(p->lo[j]) && isfinite(p->hi[j]) && p->lo[j] < p->hi[j]))
            return fail(GTMP_EINVAL, "sampling box coordinate %d: lo=%g hi=%g", j, (double)p->lo[j], (double)p->hi[j]);
    if (isnan(p->penalty) || p->penalty < 0.f) return fail(GTMP_EINVAL, "penalty must be >= 0 or +inf");
    if (isnan(p->max_edge_len) || p->max_edge_len <= 0.f) return fail(GTMP_EINVAL, "max_edge_len must be > 0 or +inf");
    const unsigned long long N = (unsigned long long)p->N;
    const unsigned long long E = N + (unsigned long long)(p->M - 1) * N * N + N * (unsigned long long)p->G;
    if (E >= (1ull << 32)) return fail(GTMP_EINVAL, "edge count %llu exceeds 2^32 - 1", E);
    const unsigned long long V = 1ull + (unsigned long long)p->M * N + (unsigned long long)p->G;
    if (V >= (1ull << 31)) return fail(GTMP_EINVAL, "vertex count too large");
    return GTMP_OK;
}

gtmp_status to_arm(const gtmp_robot *r, int d, gtmp::ArmParams *out) {
    if (r->n_joints != d) return fail(GTMP_EINVAL, "arm n_joints=%d must equal d=%d", r->n_joints, d);
    if (r->n_joints < 1 || r->n_joints > GTMP_MAX_JOINTS) return fail(GTMP_EINVAL, "n_joints=%d", r->n_joints);
    if (r->n_spheres < 1 || r->n_spheres > GTMP_MAX_ROBOT_SPHERES)
        return fail(GTMP_EINVAL, "n_spheres=%d outside 1..%d", r->n_spheres, GTMP_MAX_ROBOT_SPHERES);
    gtmp::ArmParams a{};
    a.n_joints = r->n_joints;
    a.n_spheres = r->n_spheres;
    for (int j = 0; j < r->n_joints; ++j) {
        for (int c = 0; c < 4; ++c)
            if (!isfinite(r->dh[j][c])) return fail(GTMP_EINVAL, "dh[%d][%d] not finite", j, c);
        a.a[j] = r->dh[j][0];
        a.dz[j] = r->dh[j][2];
        a.off[j] = r->dh[j][3];
        // a twist within 1e-7 rad of 0 or +-pi/2 (the FP32 pi/2 is 4.4e-8 off) is
        // taken as exact: (cos, sin)
        // = (1, 0) or (0, +-1), which the kinematics apply without products
        const double al = (double)r->dh[j][1], qt = 1.5707963267948966;
        if (fabs(al) <= 1e-7) {
            a.ca[j] = 1.f; a.sa[j] = 0.f; a.twist[j] = gtmp::kTwistNone;
        } else if (fabs(al - qt) <= 1e-7) {
            a.ca[j] = 0.f; a.sa[j] = 1.f; a.twist[j] = gtmp::kTwistPlus;
        } else if (fabs(al + qt) <= 1e-7) {
            a.ca[j] = 0.f; a.sa[j] = -1.f; a.twist[j] = gtmp::kTwistMinus;
        } else {
            a.ca[j] = (float)cos(al);
            a.sa[j] = (float)sin(al);
            a.twist[j] = gtmp::kTwistGeneral;
        }
    }
    int prev = 1;
    a.uniform_r = 1;
    a.r0 = r->sph_r[0];
    for (int k = 0; k < r->n_spheres; ++k) {
        const int L = r->sph_link[k];
        if (L < 1 || L > r->n_joints) return fail(GTMP_EINVAL, "sph_link[%d]=%d outside 1..%d", k, L, r->n_joints);
        if (L < prev) return fail(GTMP_EINVAL, "spheres must be listed in non-decreasing link order");
        prev = L;
        if (!isfinite(r->sph_t[k]) || !isfinite(r->sph_r[k]) || r->sph_r[k] < 0.f)
            return fail(GTMP_EINVAL, "sphere %d: bad t or radius", k);
        a.link[k] = L;
        a.t[k] = r->sph_t[k];
        a.tm1[k] = r->sph_t[k] - 1.f;
        a.r[k] = r->sph_r[k];
        if (r->sph_r[k] != a.r0) a.uniform_r = 0;
        a.lk_end[L - 1] = k + 1;
    }
    for (int j = 1; j < r->n_joints; ++j)  // links without spheres: empty ranges
        if (a.lk_end[j] < a.lk_end[j - 1]) a.lk_end[j] = a.lk_end[j - 1];
    // |sphere centre| <= max(1, max |t|) * sum of link lengths: frame origins
    // are at most the summed lengths sqrt(a^2 + d^2) from the base
    double len = 0.0, tmax = 1.0;
    for (int j = 0; j < r->n_joints; ++j)
        len += sqrt((double)r->dh[j][0] * r->dh[j][0] + (double)r->dh[j][2] * r->dh[j][2]);
    for (int k = 0; k < r->n_spheres; ++k) tmax = fmax(tmax, fabs((double)r->sph_t[k]));
    a.reach = (float)(len * tmax * (1.0 + 1e-6));
    a.sph_tol = 0.f;
    // per link: the spheres of link L lie on the line through o_{L-1} and
    // o_L at t, so |centre| <= |o_{L-1}| + |t| |o_L - o_{L-1}| <= (lengths of
    // links before L) + max(1, max |t|) (length of L)
    double before = 0.0;
    for (int j = 0; j < r->n_joints; ++j) {
        const double lj = sqrt((double)r->dh[j][0] * r->dh[j][0] + (double)r->dh[j][2] * r->dh[j][2]);
        double tl = 1.0;
        for (int k = 0; k < r->n_spheres; ++k)
            if (r->sph_link[k] == j + 1) tl = fmax(tl, fabs((double)r->sph_t[k]));
        a.link_reach[j] = (float)((before + tl * lj) * (1.0 + 1e-6));
        before += lj;
    }
    a.k_first = 0;
    *out = a;
    return GTMP_OK;
}

gtmp_status check_model(const gtmp_robot *robot, const gtmp_scene *scene, int d, gtmp::ArmParams *arm,
                        bool *is_arm, gtmp::SceneParams *sp) {
    if (!robot || !scene) return fail(GTMP_EINVAL, "robot or scene is NULL");
    if (scene->wdim != 2 && scene->wdim != 3) return fail(GTMP_EINVAL, "scene wdim=%d must be 2 or 3", scene->wdim);
    if (scene->n_spheres < 0 || scene->n_boxes < 0) return fail(GTMP_EINVAL, "negative obstacle count");
    if (scene->n_spheres > 0 && !scene->spheres) return fail(GTMP_EINVAL, "scene spheres is NULL");
    if (scene->n_boxes > 0 && !scene->boxes) return fail(GTMP_EINVAL, "scene boxes is NULL");
    if (robot->kind == GTMP_ROBOT_POINT) {
        if (scene->wdim != d) return fail(GTMP_EINVAL, "point robot needs wdim == d (%d vs %d)", scene->wdim, d);
        *is_arm = false;
    } else if (robot->kind == GTMP_ROBOT_DH_ARM) {
        if (scene->wdim != 3) return fail(GTMP_EINVAL, "arm needs a 3D scene");
        const gtmp_status st = to_arm(robot, d, arm);
        if (st != GTMP_OK) return st;
        *is_arm = true;
    } else {
        return fail(GTMP_EINVAL, "unknown robot kind %d", robot->kind);
    }
    sp->sph = scene->spheres;
    sp->box = scene->boxes;
    sp->n_sph = scene->n_spheres;
    sp->n_box = scene->n_boxes;
    return GTMP_OK;
}

}  // namespace

extern "C" {

const char *gtmp_status_string(gtmp_status s) {
    switch (s) {
        case GTMP_OK: return "GTMP_OK";
        case GTMP_ENOPATH: return "GTMP_ENOPATH";
        case GTMP_INCOMPLETE: return "GTMP_INCOMPLETE";
        case GTMP_EINVAL: return "GTMP_EINVAL";
        case GTMP_EHIP: return "GTMP_EHIP";
        case GTMP_EWORKSPACE: return "GTMP_EWORKSPACE";
        default: return "GTMP_UNKNOWN";
    }
}

const char *gtmp_last_error(void) { return g_err; }

const char *gtmp_version(void) { return "gtmp-gfx950 0.1"; }

gtmp_status gtmp_sample_layers(const gtmp_problem *prob, uint64_t seed, uint64_t stage, float *Q, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!Q) return fail(GTMP_EINVAL, "Q is NULL");
    return hip_status(gtmp::launch_sample_layers(*prob, seed, stage, Q, (hipStream_t)stream), "gtmp_sample_layers");
}

gtmp_status gtmp_edge_check_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_edge_plan(*prob).total;
    return GTMP_OK;
}

namespace {

// Validation and dispatch shared by the two edge-check entry points.
gtmp_status edge_check(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene, const float *q0,
                       const float *goals, const float *Q, float *C_s, float *C_h, float *C_l, float *minsd,
                       uint8_t *flags, const uint8_t *prune, void *workspace, size_t ws_bytes,
                       const gtmp_edge_opts *opts, void *stream, const char *who) {
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    gtmp_status st = check_model(robot, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (!q0 || !goals || !Q || !C_s || !C_l) return fail(GTMP_EINVAL, "q0, goals, Q, C_s and C_l must be non-NULL");
    if (prob->M > 1 && !C_h) return fail(GTMP_EINVAL, "C_h is NULL with M > 1");
    const gtmp::EdgePlan plan = gtmp::make_edge_plan(*prob);
    if (!workspace) return fail(GTMP_EINVAL, "workspace is NULL");
    if (ws_bytes < plan.total)
        return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, plan.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    gtmp_edge_opts o{};
    if (opts) o = *opts;
    if (o.mode != GTMP_CHECK_FAST && o.mode != GTMP_CHECK_FULL) return fail(GTMP_EINVAL, "unknown mode %d", o.mode);
    if (o.states_per_iter < 0 || o.states_per_iter > 8) return fail(GTMP_EINVAL, "states_per_iter=%d", o.states_per_iter);
    if (o.blocks_per_cu < 0 || o.blocks_per_cu > 32) return fail(GTMP_EINVAL, "blocks_per_cu=%d", o.blocks_per_cu);
    if (o.sphere_chunks != 0 && o.sphere_chunks != 1 && o.sphere_chunks != 2 && o.sphere_chunks != 4)
        return fail(GTMP_EINVAL, "sphere_chunks=%d (0, 1, 2 or 4)", o.sphere_chunks);
    gtmp::EdgeBuffers b{q0, goals, Q, C_s, C_h, C_l, minsd, flags, prune, workspace};
    return hip_status(gtmp::launch_edge_check(plan, is_arm ? &arm : nullptr, sp, scene->wdim, b, o, (hipStream_t)stream),
                      who);
}

}  // namespace

gtmp_status gtmp_edge_check_cost(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                                 const float *q0, const float *goals, const float *Q, float *C_s, float *C_h,
                                 float *C_l, float *minsd, uint8_t *flags, const uint8_t *prune, void *workspace,
                                 size_t ws_bytes, const gtmp_edge_opts *opts, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    return edge_check(prob, robot, scene, q0, goals, Q, C_s, C_h, C_l, minsd, flags, prune, workspace, ws_bytes, opts,
                      stream, "gtmp_edge_check_cost");
}

// ------------------------------------------------------------------ edge check without allocation
// The scratch of gtmp_edge_check_cost_noalloc: a file-scope device array,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address of each GPU's copy is looked up once per device with that
// device current and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[GTMP_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

gtmp_status scratch_addr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GTMP_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return fail(GTMP_EHIP, "scratch address not aligned");
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return GTMP_OK;
}

}  // namespace

gtmp_status gtmp_edge_check_cost_noalloc(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                                         const float *q0, const float *goals, const float *Q, float *C_s, float *C_h,
                                         float *C_l, float *minsd, uint8_t *flags, const uint8_t *prune,
                                         const gtmp_edge_opts *opts, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    const size_t need = gtmp::make_edge_plan(*prob).total;
    if (need > (size_t)GTMP_NOALLOC_SCRATCH_BYTES)
        return fail(GTMP_EINVAL, "problem needs %zu bytes of scratch; the static scratch holds %zu", need,
                    (size_t)GTMP_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    st = scratch_addr(&ws);
    if (st != GTMP_OK) return st;
    return edge_check(prob, robot, scene, q0, goals, Q, C_s, C_h, C_l, minsd, flags, prune, ws,
                      (size_t)GTMP_NOALLOC_SCRATCH_BYTES, opts, stream, "gtmp_edge_check_cost_noalloc");
}

gtmp_status gtmp_state_check(const gtmp_robot *robot, const gtmp_scene *scene, int32_t d, int64_t n, const float *X,
                             float *sd, uint8_t *coll, void *stream) {
    g_err[0] = 0;
    if (d < 1 || d > GTMP_MAX_DOF) return fail(GTMP_EINVAL, "d=%d", d);
    if (n < 0) return fail(GTMP_EINVAL, "n=%lld < 0", (long long)n);
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    gtmp_status st = check_model(robot, scene, d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (n > 0 && !X) return fail(GTMP_EINVAL, "X is NULL");
    if (!sd && !coll) return fail(GTMP_EINVAL, "sd and coll are both NULL");
    return hip_status(gtmp::launch_state_check(is_arm ? &arm : nullptr, sp, scene->wdim, d, n, X, sd, coll,
                                               (hipStream_t)stream),
                      "gtmp_state_check");
}

gtmp_status gtmp_simplify_paths(const gtmp_robot *robot, const gtmp_scene *scene, int32_t d, int32_t B, int32_t K,
                                int32_t H, const float *wp, uint8_t *valid, int32_t *idx, int32_t *count, float *cost,
                                float *out_wp, void *stream) {
    g_err[0] = 0;
    if (d < 1 || d > GTMP_MAX_DOF) return fail(GTMP_EINVAL, "d=%d", d);
    if (B < 0) return fail(GTMP_EINVAL, "B=%d < 0", B);
    if (K < 2 || K > 64) return fail(GTMP_EINVAL, "K=%d outside 2..64", K);
    if (H < 2 || H > GTMP_MAX_H) return fail(GTMP_EINVAL, "H=%d outside 2..%d", H, GTMP_MAX_H);
    if ((long long)B * K * K > (1ll << 31)) return fail(GTMP_EINVAL, "B K^2 = %lld too large", (long long)B * K * K);
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    gtmp_status st = check_model(robot, scene, d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (B > 0 && (!wp || !valid || !idx || !count || !cost)) return fail(GTMP_EINVAL, "NULL buffer");
    return hip_status(gtmp::launch_simplify(is_arm ? &arm : nullptr, sp, scene->wdim, d, B, K, H, wp, valid, idx, count,
                                            cost, out_wp, (hipStream_t)stream),
                      "gtmp_simplify_paths");
}

static gtmp_status check_rrtc(const gtmp_problem *prob, const gtmp_rrtc_opts *o) {
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!o) return fail(GTMP_EINVAL, "opts is NULL");
    if (o->budget < 1) return fail(GTMP_EINVAL, "budget=%d < 1", o->budget);
    if (o->tree_cap < 2 || o->tree_cap > 4096) return fail(GTMP_EINVAL, "tree_cap=%d outside 2..4096", o->tree_cap);
    if (gtmp::rrtc_lds_bytes(prob->d, o->tree_cap, 0) > 163840 - 8192)
        return fail(GTMP_EINVAL, "tree_cap=%d needs more than 152 KiB of LDS at d=%d", o->tree_cap, prob->d);
    if (!(o->step > 0.f) || !std::isfinite(o->step)) return fail(GTMP_EINVAL, "step must be finite and > 0");
    if (!(o->resolution > 0.f) || !std::isfinite(o->resolution))
        return fail(GTMP_EINVAL, "resolution must be finite and > 0");
    if (!(o->step / o->resolution <= 4096.f)) return fail(GTMP_EINVAL, "step / resolution > 4096");
    if (!(o->ell_factor >= 1.f) || !std::isfinite(o->ell_factor)) return fail(GTMP_EINVAL, "ell_factor must be >= 1");
    const uint64_t N = prob->N, M = prob->M, G = prob->G;
    if (N + (M - 1) * N * N + N * G >= (1ull << 32)) return fail(GTMP_EINVAL, "more than 2^32 - 1 edges");
    return GTMP_OK;
}

gtmp_status gtmp_rrtc_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_rrtc_plan(*prob).total;
    return GTMP_OK;
}

gtmp_status gtmp_rrtc_repair(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                             const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                             uint8_t *flags, uint64_t seed, uint64_t stage, const gtmp_rrtc_opts *opts,
                             void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_rrtc(prob, opts);
    if (st != GTMP_OK) return st;
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    st = check_model(robot, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (!q0 || !goals || !Q || !C_s || !C_l || !flags || !workspace) return fail(GTMP_EINVAL, "NULL buffer");
    if (prob->M > 1 && !C_h) return fail(GTMP_EINVAL, "C_h is NULL with M > 1");
    const size_t need = gtmp::make_rrtc_plan(*prob).total;
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    return hip_status(gtmp::launch_rrtc_repair(*prob, is_arm ? &arm : nullptr, sp, scene->wdim, q0, goals, Q, C_s, C_h,
                                               C_l, flags, seed, stage, *opts, workspace, (hipStream_t)stream),
                      "gtmp_rrtc_repair");
}

gtmp_status gtmp_rrtc_local_path(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                                 const float *q0, const float *goals, const float *Q, uint64_t edge, uint64_t seed,
                                 uint64_t stage, const gtmp_rrtc_opts *opts, float *path, int32_t *count, float *cost,
                                 void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_rrtc(prob, opts);
    if (st != GTMP_OK) return st;
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    st = check_model(robot, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    const uint64_t N = prob->N, M = prob->M, G = prob->G;
    if (edge >= N + (M - 1) * N * N + N * G) return fail(GTMP_EINVAL, "edge %llu out of range", (unsigned long long)edge);
    if (!q0 || !goals || !Q || !path || !count || !cost) return fail(GTMP_EINVAL, "NULL buffer");
    return hip_status(gtmp::launch_rrtc_path(*prob, is_arm ? &arm : nullptr, sp, scene->wdim, q0, goals, Q, edge, seed,
                                             stage, *opts, path, count, cost, (hipStream_t)stream),
                      "gtmp_rrtc_local_path");
}

gtmp_status gtmp_lazy_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_lazy_plan(*prob).total;
    return GTMP_OK;
}

gtmp_status gtmp_plan_lazy(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                           const float *q0, const float *goals, const float *Q, float *C_s, float *C_h, float *C_l,
                           uint8_t *flags, float *V, int32_t *A, float *V_s, int32_t *a_s, int32_t *idx, float *wp,
                           float *cost, float band, int32_t max_rounds, unsigned long long *stats, int32_t *rounds,
                           void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    st = check_model(robot, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (!(band >= 0.f) || !std::isfinite(band)) return fail(GTMP_EINVAL, "band must be finite and >= 0");
    if (max_rounds < 1) return fail(GTMP_EINVAL, "max_rounds=%d < 1", max_rounds);
    if (!q0 || !goals || !Q || !C_s || !C_l || !flags || !V || !A || !V_s || !a_s || !idx || !wp || !cost ||
        !workspace)
        return fail(GTMP_EINVAL, "NULL buffer");
    if (prob->M > 1 && !C_h) return fail(GTMP_EINVAL, "C_h is NULL with M > 1");
    const size_t need = gtmp::make_lazy_plan(*prob).total;
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    gtmp_edge_opts eo{};
    if (edge_opts) eo = *edge_opts;
    int r = 0;
    bool done = false;
    st = hip_status(gtmp::launch_plan_lazy(*prob, is_arm ? &arm : nullptr, sp, scene->wdim, q0, goals, Q, C_s, C_h, C_l,
                                           flags, V, A, V_s, a_s, idx, wp, cost, band, max_rounds, stats, eo,
                                           workspace, &r, &done, (hipStream_t)stream),
                    "gtmp_plan_lazy");
    if (st != GTMP_OK) return st;
    if (rounds) *rounds = r;
    return done ? GTMP_OK : GTMP_INCOMPLETE;
}

gtmp_status gtmp_minplus_sweep(int32_t M, int32_t N, int32_t G, const float *C_s, const float *C_h, const float *C_l,
                               const float *Vg, float *V, int32_t *A, float *V_s, int32_t *a_s, void *stream) {
    g_err[0] = 0;
    if (M < 1 || N < 1 || G < 1) return fail(GTMP_EINVAL, "M=%d N=%d G=%d must be >= 1", M, N, G);
    if ((long long)(M - 1) * N * (long long)N >= (1ll << 40)) return fail(GTMP_EINVAL, "C_h too large");
    if (!C_s || !C_l || !V || !A || !V_s || !a_s) return fail(GTMP_EINVAL, "NULL buffer");
    if (M > 1 && !C_h) return fail(GTMP_EINVAL, "C_h is NULL with M > 1");
    return hip_status(gtmp::launch_minplus(M, N, G, C_s, C_h, C_l, Vg, V, A, V_s, a_s, (hipStream_t)stream),
                      "gtmp_minplus_sweep");
}

gtmp_status gtmp_extract_path(int32_t M, int32_t N, int32_t G, int32_t d, const int32_t *a_s, const int32_t *A,
                              const float *V_s, const float *Q, const float *q0, const float *goals, int32_t *idx,
                              float *wp, float *cost, void *stream) {
    g_err[0] = 0;
    if (M < 1 || N < 1 || G < 1 || d < 1 || d > GTMP_MAX_DOF) return fail(GTMP_EINVAL, "bad sizes");
    if (!a_s || !A || !V_s || !Q || !q0 || !goals || !idx || !wp || !cost) return fail(GTMP_EINVAL, "NULL buffer");
    return hip_status(gtmp::launch_extract(M, N, G, d, a_s, A, V_s, Q, q0, goals, idx, wp, cost, (hipStream_t)stream),
                      "gtmp_extract_path");
}

gtmp_status gtmp_expand_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    const uint64_t G = (uint64_t)prob->G, N = (uint64_t)prob->N;
    if (N * (N > G ? N : G) >= (1ull << 32)) return fail(GTMP_EINVAL, "too many sample pairs");
    *bytes = gtmp::make_expand_plan(*prob).total;
    return GTMP_OK;
}

gtmp_status gtmp_expand_samples(const gtmp_problem *prob, const float *q0, const float *goals, const float *Q_old,
                                int32_t n_old, float *Q_new, const float *c_best, uint64_t seed, uint64_t stage,
                                void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    size_t need = 0;
    gtmp_status st = gtmp_expand_workspace_size(prob, &need);
    if (st != GTMP_OK) return st;
    if (n_old < 0 || n_old > prob->N) return fail(GTMP_EINVAL, "n_old=%d outside 0..N", n_old);
    if (!q0 || !goals || !Q_new || !c_best || !workspace) return fail(GTMP_EINVAL, "NULL buffer");
    if (n_old > 0 && !Q_old) return fail(GTMP_EINVAL, "Q_old is NULL with n_old > 0");
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    if (n_old > 0) {
        const char *a = reinterpret_cast<const char *>(Q_old), *b = reinterpret_cast<const char *>(Q_new);
        const size_t la = sizeof(float) * (size_t)prob->M * n_old * prob->d, lb = sizeof(float) * (size_t)prob->M * prob->N * prob->d;
        if (a < b + lb && b < a + la) return fail(GTMP_EINVAL, "Q_old and Q_new overlap");
    }
    return hip_status(gtmp::launch_expand(*prob, q0, goals, Q_old, n_old, Q_new, c_best, seed, stage, workspace,
                                          (hipStream_t)stream),
                      "gtmp_expand_samples");
}

gtmp_status gtmp_sample_informed(const gtmp_problem *prob, const float *q0, const float *goals, const float *c_best,
                                 uint64_t seed, uint64_t stage, int32_t m, int32_t count, float *X, int32_t *attempts,
                                 void *workspace, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (count < 0 || m < 0) return fail(GTMP_EINVAL, "count and m must be >= 0");
    if (!q0 || !goals || !c_best || !workspace || (count > 0 && !X)) return fail(GTMP_EINVAL, "NULL buffer");
    return hip_status(gtmp::launch_informed_batch(*prob, q0, goals, c_best, seed, stage, (uint32_t)m, count, X,
                                                  attempts, workspace, (hipStream_t)stream),
                      "gtmp_sample_informed");
}

static gtmp_status check_net(const gtmp_surrogate *net, bool writable, gtmp::SurNet *out);

gtmp_status gtmp_expand_biased_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = gtmp_expand_workspace_size(prob, bytes);
    if (st != GTMP_OK) return st;
    *bytes = gtmp::make_expand_plan(*prob, true).total;
    return GTMP_OK;
}

gtmp_status gtmp_expand_samples_biased(const gtmp_problem *prob, const float *q0, const float *goals,
                                       const float *Q_old, int32_t n_old, float *Q_new, const float *c_best,
                                       uint64_t seed, uint64_t stage, const gtmp_surrogate *net, float tau_logit,
                                       void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    size_t need = 0;
    gtmp_status st = gtmp_expand_biased_workspace_size(prob, &need);
    if (st != GTMP_OK) return st;
    gtmp::SurNet sn{};
    st = check_net(net, false, &sn);
    if (st != GTMP_OK) return st;
    if (net->d != prob->d) return fail(GTMP_EINVAL, "net d=%d differs from problem d=%d", net->d, prob->d);
    if (n_old < 0 || n_old > prob->N) return fail(GTMP_EINVAL, "n_old=%d outside 0..N", n_old);
    if (!q0 || !goals || !Q_new || !c_best || !workspace) return fail(GTMP_EINVAL, "NULL buffer");
    if (n_old > 0 && !Q_old) return fail(GTMP_EINVAL, "Q_old is NULL with n_old > 0");
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    if (n_old > 0) {
        const char *a = reinterpret_cast<const char *>(Q_old), *b = reinterpret_cast<const char *>(Q_new);
        const size_t la = sizeof(float) * (size_t)prob->M * n_old * prob->d, lb = sizeof(float) * (size_t)prob->M * prob->N * prob->d;
        if (a < b + lb && b < a + la) return fail(GTMP_EINVAL, "Q_old and Q_new overlap");
    }
    return hip_status(gtmp::launch_expand(*prob, q0, goals, Q_old, n_old, Q_new, c_best, seed, stage, workspace,
                                          (hipStream_t)stream, &sn, tau_logit),
                      "gtmp_expand_samples_biased");
}

static gtmp_status check_anytime(const gtmp_problem *prob, const gtmp_anytime_opts *o) {
    if (!o) return fail(GTMP_EINVAL, "opts is NULL");
    if (o->max_stages < 1) return fail(GTMP_EINVAL, "max_stages=%d < 1", o->max_stages);
    if (o->simplify) {
        const int Mx = o->mode == GTMP_ANYTIME_GROWING ? o->M_max : prob->M;
        if (Mx + 2 > 64) return fail(GTMP_EINVAL, "simplify needs at most 64 waypoints (M=%d)", Mx);
    }
    if (o->lp) {
        gtmp_problem big = *prob;
        if (o->mode == GTMP_ANYTIME_GROWING) {
            big.M = o->M_max > 0 ? o->M_max : prob->M;
            big.N = o->N_max > 0 ? o->N_max : prob->N;
        }
        gtmp_status st = check_rrtc(&big, o->lp);
        if (st != GTMP_OK) return st;
    }
    if (o->mode == GTMP_ANYTIME_RESTART) return check_problem(prob);
    if (o->mode != GTMP_ANYTIME_GROWING) return fail(GTMP_EINVAL, "unknown anytime mode %d", o->mode);
    if (o->M_min < 1 || o->M_min > o->M_max) return fail(GTMP_EINVAL, "need 1 <= M_min <= M_max");
    if (o->N_min < 1 || o->N_min > o->N_max) return fail(GTMP_EINVAL, "need 1 <= N_min <= N_max");
    gtmp_problem big = *prob;
    big.M = o->M_max;
    big.N = o->N_max;
    gtmp_status st = check_problem(&big);
    if (st != GTMP_OK) return st;
    size_t tmp = 0;
    st = gtmp_expand_workspace_size(&big, &tmp);
    if (st != GTMP_OK) return st;
    if (o->bias_net) {
        gtmp::SurNet sn{};
        st = check_net(o->bias_net, false, &sn);
        if (st != GTMP_OK) return st;
        if (o->bias_net->d != prob->d) return fail(GTMP_EINVAL, "bias net d=%d differs from d=%d", o->bias_net->d, prob->d);
    }
    return GTMP_OK;
}

gtmp_status gtmp_anytime_workspace_size(const gtmp_problem *prob, const gtmp_anytime_opts *opts, size_t *bytes) {
    g_err[0] = 0;
    if (!prob) return fail(GTMP_EINVAL, "problem is NULL");
    gtmp_status st = check_anytime(prob, opts);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_anytime_plan(*prob, *opts).total;
    return GTMP_OK;
}

gtmp_status gtmp_plan_anytime(const gtmp_problem *prob, const gtmp_robot *robot, const gtmp_scene *scene,
                              const float *q0, const float *goals, uint64_t seed, const gtmp_anytime_opts *opts,
                              float *best_cost, int32_t *best_idx, float *best_wp, int32_t *best_meta,
                              float *stage_costs, void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts,
                              void *stream) {
    g_err[0] = 0;
    size_t need = 0;
    gtmp_status st = gtmp_anytime_workspace_size(prob, opts, &need);
    if (st != GTMP_OK) return st;
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    st = check_model(robot, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (!q0 || !goals || !best_cost || !best_idx || !best_wp || !best_meta || !stage_costs || !workspace)
        return fail(GTMP_EINVAL, "NULL buffer");
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    gtmp_edge_opts eo{};
    if (edge_opts) eo = *edge_opts;
    if (eo.mode != GTMP_CHECK_FAST && eo.mode != GTMP_CHECK_FULL) return fail(GTMP_EINVAL, "unknown edge mode");
    gtmp::AnytimeOut out{best_cost, best_idx, best_wp, best_meta, stage_costs};
    gtmp::SurNet sn{};
    const bool biased = opts->mode == GTMP_ANYTIME_GROWING && opts->bias_net;
    if (biased) (void)check_net(opts->bias_net, false, &sn);
    return hip_status(gtmp::launch_anytime(*prob, is_arm ? &arm : nullptr, sp, scene->wdim, q0, goals, seed, *opts, eo,
                                           out, workspace, (hipStream_t)stream, biased ? &sn : nullptr),
                      "gtmp_plan_anytime");
}

gtmp_status gtmp_batch_workspace_size(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts,
                                      size_t *bytes);

static gtmp_status check_batch(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts,
                               std::vector<gtmp::ArmParams> *arms) {
    if (!plans || n < 1) return fail(GTMP_EINVAL, "need at least one plan");
    if (!opts) return fail(GTMP_EINVAL, "opts is NULL");
    if ((opts->sphere_chunks != 0 && opts->sphere_chunks != 1 && opts->sphere_chunks != 2 && opts->sphere_chunks != 4) ||
        opts->states_per_iter < 0 || opts->states_per_iter > 8 ||
        opts->blocks_per_cu < 0 || opts->blocks_per_cu > 32)
        return fail(GTMP_EINVAL, "bad batch options");
    arms->assign(n, gtmp::ArmParams{});
    for (int p = 0; p < n; ++p) {
        const gtmp_plan_desc &D = plans[p];
        gtmp_status st = check_problem(&D.problem);
        if (st != GTMP_OK) return fail(st, "plan %d: %s", p, g_err);
        gtmp::SceneParams sp{};
        bool is_arm = false;
        st = check_model(&D.robot, &D.scene, D.problem.d, &(*arms)[p], &is_arm, &sp);
        if (st != GTMP_OK) return fail(st, "plan %d: %s", p, g_err);
        if (!D.q0 || !D.goals) return fail(GTMP_EINVAL, "plan %d: q0 or goals is NULL", p);
        if (D.stages < 1) return fail(GTMP_EINVAL, "plan %d: stages < 1", p);
        if (D.mode == GTMP_ANYTIME_GROWING) {
            if (D.M_min < 1 || D.M_min > D.problem.M || D.N_min < 1 || D.N_min > D.problem.N)
                return fail(GTMP_EINVAL, "plan %d: need 1 <= M_min <= M and 1 <= N_min <= N", p);
            size_t tmp = 0;
            st = gtmp_expand_workspace_size(&D.problem, &tmp);
            if (st != GTMP_OK) return fail(st, "plan %d: %s", p, g_err);
        } else if (D.mode != GTMP_ANYTIME_RESTART) {
            return fail(GTMP_EINVAL, "plan %d: unknown mode %d", p, D.mode);
        }
    }
    return GTMP_OK;
}

gtmp_status gtmp_batch_workspace_size(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts,
                                      size_t *bytes) {
    g_err[0] = 0;
    std::vector<gtmp::ArmParams> arms;
    gtmp_status st = check_batch(plans, n, opts, &arms);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_batch_layout(plans, n, *opts).total;
    return GTMP_OK;
}

gtmp_status gtmp_plan_batch(const gtmp_plan_desc *plans, int32_t n, const gtmp_batch_opts *opts, float *best_cost,
                            int32_t *best_idx, float *best_wp, int32_t *best_meta, float *stage_costs,
                            int32_t stage_stride, void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    std::vector<gtmp::ArmParams> arms;
    gtmp_status st = check_batch(plans, n, opts, &arms);
    if (st != GTMP_OK) return st;
    if (!best_cost || !best_idx || !best_wp || !best_meta || !stage_costs || !workspace)
        return fail(GTMP_EINVAL, "NULL buffer");
    const gtmp::BatchLayout L = gtmp::make_batch_layout(plans, n, *opts);
    if (stage_stride < L.max_stages) return fail(GTMP_EINVAL, "stage_stride=%d < %d stages", stage_stride, L.max_stages);
    if (ws_bytes < L.total) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    gtmp::BatchOut out;
    out.best_cost = best_cost;
    out.best_idx = best_idx;
    out.best_wp = best_wp;
    out.best_meta = best_meta;
    out.stage_costs = stage_costs;
    out.stage_stride = stage_stride;
    out.stats = opts->stats;
    out.idx_offset.resize(n);
    out.wp_offset.resize(n);
    size_t io = 0, wo = 0;
    for (int p = 0; p < n; ++p) {
        out.idx_offset[p] = io;
        out.wp_offset[p] = wo;
        io += (size_t)plans[p].problem.M + 1;
        wo += (size_t)(plans[p].problem.M + 2) * plans[p].problem.d;
    }
    return hip_status(gtmp::launch_batch(plans, arms.data(), n, *opts, L, out, workspace, (hipStream_t)stream),
                      "gtmp_plan_batch");
}

// ------------------------------------------------------------------ a9 surrogate
static gtmp_status check_net(const gtmp_surrogate *net, bool writable, gtmp::SurNet *out) {
    if (!net) return fail(GTMP_EINVAL, "net is NULL");
    if (net->d < 1 || net->d > GTMP_MAX_DOF) return fail(GTMP_EINVAL, "net d=%d outside 1..%d", net->d, GTMP_MAX_DOF);
    if (!net->fourier || !net->params || !net->params_bf16) return fail(GTMP_EINVAL, "net has a NULL buffer");
    if ((reinterpret_cast<uintptr_t>(net->params_bf16) & 15) != 0 || (reinterpret_cast<uintptr_t>(net->params) & 15) != 0)
        return fail(GTMP_EINVAL, "params and params_bf16 must be 16-byte aligned");
    (void)writable;
    out->d = net->d;
    out->fourier = net->fourier;
    out->p32 = net->params;
    out->p16 = net->params_bf16;
    return GTMP_OK;
}

static gtmp_status check_ws(void *workspace, size_t ws_bytes, size_t need) {
    if (!workspace) return fail(GTMP_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    return GTMP_OK;
}

gtmp_status gtmp_surrogate_layout(int32_t offsets[11]) {
    g_err[0] = 0;
    if (!offsets) return fail(GTMP_EINVAL, "offsets is NULL");
    const gtmp::SurLayout L = gtmp::sur_layout();
    for (int l = 0; l < 4; ++l) {
        offsets[2 * l] = L.W[l];
        offsets[2 * l + 1] = L.b[l];
    }
    offsets[8] = L.w5;
    offsets[9] = L.b5;
    offsets[10] = L.total;
    return GTMP_OK;
}

gtmp_status gtmp_surrogate_refresh_bf16(const gtmp_surrogate *net, void *stream) {
    g_err[0] = 0;
    gtmp::SurNet sn{};
    gtmp_status st = check_net(net, true, &sn);
    if (st != GTMP_OK) return st;
    return hip_status(gtmp::launch_sur_refresh(sn, (hipStream_t)stream), "gtmp_surrogate_refresh_bf16");
}

gtmp_status gtmp_surrogate_workspace_size(int64_t n, size_t *bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    if (n < 1 || n > (1ll << 30)) return fail(GTMP_EINVAL, "n=%lld outside 1..2^30", (long long)n);
    const int64_t rows = (n + 255) / 256 * 256;
    *bytes = gtmp::sur_workspace_bytes(rows);
    return GTMP_OK;
}

gtmp_status gtmp_surrogate_infer(const gtmp_surrogate *net, int64_t n, const float *X, float *logits, void *workspace,
                                 size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    gtmp::SurNet sn{};
    gtmp_status st = check_net(net, false, &sn);
    if (st != GTMP_OK) return st;
    if (n < 0) return fail(GTMP_EINVAL, "n=%lld < 0", (long long)n);
    if (n == 0) return GTMP_OK;
    if (!X || !logits) return fail(GTMP_EINVAL, "NULL buffer");
    st = check_ws(workspace, ws_bytes, gtmp::sur_infer_bytes(256));
    if (st != GTMP_OK) return st;
    return hip_status(gtmp::launch_sur_infer(sn, n, X, logits, workspace, ws_bytes, (hipStream_t)stream),
                      "gtmp_surrogate_infer");
}

gtmp_status gtmp_surrogate_grad(const gtmp_surrogate *net, int32_t n, const float *X, const uint8_t *y, float *grad,
                                float *loss, float *logits, void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    gtmp::SurNet sn{};
    gtmp_status st = check_net(net, false, &sn);
    if (st != GTMP_OK) return st;
    if (n < 256 || n % 256 != 0) return fail(GTMP_EINVAL, "n=%d must be a positive multiple of 256", n);
    if (!X || !y || !grad || !loss) return fail(GTMP_EINVAL, "NULL buffer");
    st = check_ws(workspace, ws_bytes, gtmp::sur_workspace_bytes(n));
    if (st != GTMP_OK) return st;
    return hip_status(gtmp::launch_sur_grad(sn, n, X, y, grad, loss, logits, workspace, (hipStream_t)stream),
                      "gtmp_surrogate_grad");
}

gtmp_status gtmp_surrogate_adam(const gtmp_surrogate *net, const float *grad, float *m, float *v, int32_t t, float lr,
                                float beta1, float beta2, float eps, void *stream) {
    g_err[0] = 0;
    gtmp::SurNet sn{};
    gtmp_status st = check_net(net, true, &sn);
    if (st != GTMP_OK) return st;
    if (!grad || !m || !v) return fail(GTMP_EINVAL, "NULL buffer");
    if (t < 1) return fail(GTMP_EINVAL, "t=%d < 1", t);
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(GTMP_EINVAL, "bad Adam hyper-parameters");
    return hip_status(gtmp::launch_sur_adam(sn, grad, m, v, t, lr, beta1, beta2, eps, (hipStream_t)stream),
                      "gtmp_surrogate_adam");
}

gtmp_status gtmp_surrogate_label_states(const gtmp_problem *prob, uint64_t seed, uint64_t stage, int64_t n, float *X,
                                        void *stream) {
    g_err[0] = 0;
    if (!prob) return fail(GTMP_EINVAL, "problem is NULL");
    gtmp_problem q = *prob;  // only d, the box and H are used
    q.M = 1;
    q.N = 1;
    q.G = 1;
    gtmp_status st = check_problem(&q);
    if (st != GTMP_OK) return st;
    if (prob->H < 3) return fail(GTMP_EINVAL, "H=%d: label states need interior states (H >= 3)", prob->H);
    if (n < 0 || n > (1ll << 31) - 1) return fail(GTMP_EINVAL, "n=%lld outside 0..2^31-1", (long long)n);
    if (n > 0 && !X) return fail(GTMP_EINVAL, "X is NULL");
    return hip_status(gtmp::launch_sur_label_states(*prob, seed, stage, n, X, (hipStream_t)stream),
                      "gtmp_surrogate_label_states");
}

gtmp_status gtmp_surrogate_prune_workspace_size(const gtmp_problem *prob, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::sur_prune_bytes(*prob);
    return GTMP_OK;
}

gtmp_status gtmp_surrogate_prune(const gtmp_problem *prob, const gtmp_surrogate *net, const float *q0,
                                 const float *goals, const float *Q, const uint8_t *vcoll, float tau_logit,
                                 uint8_t *prune, float *logits, void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    gtmp::SurNet sn{};
    st = check_net(net, false, &sn);
    if (st != GTMP_OK) return st;
    if (net->d != prob->d) return fail(GTMP_EINVAL, "net d=%d differs from problem d=%d", net->d, prob->d);
    if (!q0 || !goals || !Q || !prune) return fail(GTMP_EINVAL, "NULL buffer");
    if (isnan(tau_logit)) return fail(GTMP_EINVAL, "tau_logit is NaN");
    st = check_ws(workspace, ws_bytes, gtmp::sur_prune_bytes(*prob));
    if (st != GTMP_OK) return st;
    return hip_status(gtmp::launch_sur_prune(*prob, sn, q0, goals, Q, vcoll, tau_logit, prune, logits, workspace,
                                             (hipStream_t)stream),
                      "gtmp_surrogate_prune");
}

gtmp_status gtmp_surrogate_threshold_workspace_size(size_t *bytes) {
    g_err[0] = 0;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::sur_threshold_bytes();
    return GTMP_OK;
}

gtmp_status gtmp_surrogate_threshold(const float *logits, const uint8_t *flags, int64_t E, double recall, float *tau,
                                     void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    if (E < 0) return fail(GTMP_EINVAL, "E=%lld is negative", (long long)E);
    if (!(recall > 0.0 && recall <= 1.0)) return fail(GTMP_EINVAL, "recall=%g outside (0, 1]", recall);
    if (!tau || (E > 0 && (!logits || !flags))) return fail(GTMP_EINVAL, "NULL buffer");
    gtmp_status st = check_ws(workspace, ws_bytes, gtmp::sur_threshold_bytes());
    if (st != GTMP_OK) return st;
    return hip_status(gtmp::launch_sur_threshold(logits, flags, E, recall, tau, workspace, (hipStream_t)stream),
                      "gtmp_surrogate_threshold");
}

// ------------------------------------------------------------------ class-augmented sweep
static gtmp_status check_class_sizes(int M, int N, int G, int L, int k) {
    if (M < 1 || M > 126) return fail(GTMP_EINVAL, "class sweep needs 1 <= M <= 126 (labels of at most 127 edges)");
    if (N < 1 || N >= (1 << 24) || G < 1 || G >= (1 << 24)) return fail(GTMP_EINVAL, "N=%d G=%d out of range", N, G);
    if (L < 1 || L > 64) return fail(GTMP_EINVAL, "L=%d outside 1..64", L);
    if (k < 0 || k > 16) return fail(GTMP_EINVAL, "k=%d outside 0..16 representative points", k);
    return GTMP_OK;
}

gtmp_status gtmp_class_sweep_workspace_size(int32_t M, int32_t N, int32_t L, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_class_sizes(M, N, 1, L, 0);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_class_plan(M, N, L).total;
    return GTMP_OK;
}

gtmp_status gtmp_class_sweep(int32_t M, int32_t N, int32_t G, int32_t L, const float *Q, const float *q0,
                             const float *goals, const float *C_s, const float *C_h, const float *C_l, float penalty,
                             const float *reps, int32_t k, uint64_t *labels, float *costs, int32_t *chains,
                             int32_t *count, uint32_t *overflow, void *workspace, size_t ws_bytes, void *stream) {
    g_err[0] = 0;
    gtmp_status st = check_class_sizes(M, N, G, L, k);
    if (st != GTMP_OK) return st;
    if (!Q || !q0 || !goals || !C_s || !C_l || !labels || !costs || !chains || !count || !overflow || !workspace ||
        (k > 0 && !reps) || (M > 1 && !C_h))
        return fail(GTMP_EINVAL, "NULL buffer");
    if (!(penalty > 0.f)) return fail(GTMP_EINVAL, "penalty must be > 0");
    const size_t need = gtmp::make_class_plan(M, N, L).total;
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    return hip_status(gtmp::launch_class_sweep(M, N, G, L, Q, q0, goals, C_s, C_h, C_l, penalty, reps, k, labels, costs,
                                               chains, count, overflow, true, workspace, (hipStream_t)stream),
                      "gtmp_class_sweep");
}

gtmp_status gtmp_class_anytime_workspace_size(const gtmp_problem *prob, int32_t L, size_t *bytes) {
    g_err[0] = 0;
    gtmp_status st = check_problem(prob);
    if (st != GTMP_OK) return st;
    if (prob->d != 2) return fail(GTMP_EINVAL, "class archive needs d = 2");
    st = check_class_sizes(prob->M, prob->N, prob->G, L, 0);
    if (st != GTMP_OK) return st;
    if (!bytes) return fail(GTMP_EINVAL, "bytes is NULL");
    *bytes = gtmp::make_class_anytime_plan(*prob, L).total;
    return GTMP_OK;
}

gtmp_status gtmp_plan_classes(const gtmp_problem *prob, const gtmp_scene *scene, const float *q0, const float *goals,
                              uint64_t seed, int32_t stages, const float *reps, int32_t k, int32_t L, int32_t cap,
                              uint64_t *a_labels, float *a_costs, int32_t *a_stage, float *a_wp, int32_t *a_count,
                              uint32_t *overflow, void *workspace, size_t ws_bytes, const gtmp_edge_opts *edge_opts,
                              void *stream) {
    g_err[0] = 0;
    size_t need = 0;
    gtmp_status st = gtmp_class_anytime_workspace_size(prob, L, &need);
    if (st != GTMP_OK) return st;
    st = check_class_sizes(prob->M, prob->N, prob->G, L, k);
    if (st != GTMP_OK) return st;
    gtmp::ArmParams arm{};
    gtmp::SceneParams sp{};
    bool is_arm = false;
    gtmp_robot point{};
    point.kind = GTMP_ROBOT_POINT;
    st = check_model(&point, scene, prob->d, &arm, &is_arm, &sp);
    if (st != GTMP_OK) return st;
    if (scene->wdim != 2) return fail(GTMP_EINVAL, "class archive needs a 2D scene");
    if (stages < 1) return fail(GTMP_EINVAL, "stages=%d < 1", stages);
    if (cap < 1) return fail(GTMP_EINVAL, "cap=%d < 1", cap);
    if (!q0 || !goals || !a_labels || !a_costs || !a_stage || !a_wp || !a_count || !overflow || !workspace ||
        (k > 0 && !reps))
        return fail(GTMP_EINVAL, "NULL buffer");
    if (ws_bytes < need) return fail(GTMP_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return fail(GTMP_EINVAL, "workspace must be 256-byte aligned");
    gtmp_edge_opts eo{};
    if (edge_opts) eo = *edge_opts;
    eo.mode = GTMP_CHECK_FAST;
    return hip_status(gtmp::launch_plan_classes(*prob, sp, q0, goals, seed, stages, reps, k, L, cap, a_labels, a_costs,
                                                a_stage, a_wp, a_count, overflow, eo, workspace, (hipStream_t)stream),
                      "gtmp_plan_classes");
}

}  // extern "C"

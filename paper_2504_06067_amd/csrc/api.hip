// C-ABI entry points of libnsga3: host-side validation, workspace carving and
// the ordered enqueue of each stage's kernels. No call allocates memory or
// waits for the device, except nsga3_read_status (which waits by design).
#include <string.h>

#include "nsga3_internal.h"

namespace nsga3 {

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout make_layout(int M, int m, int H, int N) {
    Layout L;
    L.M = M; L.m = m; L.H = H; L.N = N;
    L.Mp = (M + 63) / 64 * 64;
    L.W = L.Mp / 64;
    L.Hp = (H + 15) / 16 * 16;
    const size_t Mp = (size_t)L.Mp, W = (size_t)L.W, Hp = (size_t)L.Hp;
    size_t o = 0;
    auto take = [&o](size_t bytes) { size_t at = o; o += up256(bytes); return at; };
    L.ctrl = take(4096);
    L.ft = take((size_t)m * Mp * 4);
    L.nd = take(Mp * 4);
    L.mask = take(W * Mp * 8);
    L.rowm = take(W * Mp * 8);
    L.wit = take(Mp * 4);
    // alive ring: ns slots of W words, one 128-byte line per word
    L.ns = (int)((64ull << 20) / (W * 128));
    if (L.ns > 254) L.ns = 254;
    if (L.ns < 8) L.ns = 8;
    L.alive = take((size_t)L.ns * W * 128);
    L.facc = take(3 * 33 * 32 * 8);  // front-peeling counter ring
    L.list = take(Mp * 4);
    L.fn = take(Mp * (size_t)m * 4);
    L.rank = take(Mp * 4);
    L.pi = take(Mp * 4);
    L.dist = take(Mp * 4);
    L.akey = take(Mp * 8);
    L.wn = take((size_t)m * Hp * 4);
    L.rho = take(Hp * 4);
    L.cnt = take(Hp * 4);
    L.off = take((Hp + 1) * 4);
    L.fill = take(Hp * 4);
    L.tpick = take(Hp * 4);
    L.members = take(Mp * 4);
    L.picked = take(Mp * 4);
    L.remain = take((W + (size_t)H + 2) * 8);
    L.tiles = take(((size_t)(M + 4095) / 4096 + 1) * 4);
    L.total = o;
    return L;
}

Ptrs carve(const Layout &L, void *ws) {
    char *b = (char *)ws;
    Ptrs P;
    P.ctrl = (Ctrl *)(b + L.ctrl);
    P.ft = (float *)(b + L.ft);
    P.nd = (int *)(b + L.nd);
    P.mask = (u64 *)(b + L.mask);
    P.rowm = (u64 *)(b + L.rowm);
    P.wit = (int *)(b + L.wit);
    P.alive = (u64 *)(b + L.alive);
    P.facc = (u64 *)(b + L.facc);
    P.list = (int *)(b + L.list);
    P.fn = (float *)(b + L.fn);
    P.rank = (int *)(b + L.rank);
    P.pi = (int *)(b + L.pi);
    P.dist = (float *)(b + L.dist);
    P.akey = (u64 *)(b + L.akey);
    P.wn = (float *)(b + L.wn);
    P.rho = (int *)(b + L.rho);
    P.cnt = (int *)(b + L.cnt);
    P.off = (int *)(b + L.off);
    P.fill = (int *)(b + L.fill);
    P.tpick = (int *)(b + L.tpick);
    P.members = (int *)(b + L.members);
    P.picked = (int *)(b + L.picked);
    P.remain = (u64 *)(b + L.remain);
    P.tiles = (int *)(b + L.tiles);
    return P;
}

Dev device_info() {
    static int cached_cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cached_cus[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached_cus[dev] = cus;
    }
    return Dev{cached_cus[dev]};
}

static bool valid_shape(int M, int m, int H, int N) {
    return M >= 2 && M <= NSGA3_MAX_POINTS && m >= 2 && m <= NSGA3_MAX_OBJECTIVES && H >= 1 &&
           H <= NSGA3_MAX_POINTS && N >= 1 && N <= M;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

static int check_ws(const Layout &L, const void *ws, size_t ws_bytes) {
    if (!ws || !aligned(ws, 256)) return NSGA3_EINVAL;
    if (ws_bytes < L.total) return NSGA3_EWORKSPACE;
    return NSGA3_OK;
}

static int to_status(hipError_t e) { return e == hipSuccess ? NSGA3_OK : NSGA3_EHIP; }

// ---------------------------------------------------------- instrumentation

namespace {
constexpr int PROF_POOL = 8192;   // event pairs per enable
constexpr int PROF_NAMES = 64;
struct ProfState {
    bool on = false;
    bool all = false;
    char filter[512] = {0};
    hipEvent_t ev[2 * PROF_POOL];
    const char *rec_name[PROF_POOL];
    int used = 0, created = 0, dropped = 0;
};
ProfState g_prof;

bool prof_wanted(const char *name) {
    if (!g_prof.on) return false;
    if (g_prof.all) return true;
    // comma-separated exact names
    const size_t n = strlen(name);
    const char *f = g_prof.filter;
    while (*f) {
        const char *e = strchr(f, ',');
        const size_t len = e ? (size_t)(e - f) : strlen(f);
        if (len == n && strncmp(f, name, n) == 0) return true;
        if (!e) break;
        f = e + 1;
    }
    return false;
}
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t s) : slot(-1), stream(s) {
    if (!prof_wanted(name)) return;
    if (g_prof.used >= g_prof.created) { ++g_prof.dropped; return; }
    slot = g_prof.used++;
    g_prof.rec_name[slot] = name;
    if (hipEventRecord(g_prof.ev[2 * slot], s) != hipSuccess) slot = -1;
}

ProfScope::~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], stream);
}

}  // namespace nsga3

using namespace nsga3;

extern "C" {

size_t nsga3_workspace_bytes(int32_t M, int32_t m, int32_t H, int32_t N) {
    if (!valid_shape(M, m, H, N)) return 0;
    return make_layout(M, m, H, N).total;
}

int nsga3_nd_sort(const float *F, int32_t M, int32_t m, int32_t n_stop, int32_t *rank,
                  int32_t *front_info, void *ws, size_t ws_bytes, void *stream) {
    if (!F || !rank || !front_info || !valid_shape(M, m, 1, 1) || !aligned(F, 4) ||
        !aligned(rank, 4) || !aligned(front_info, 4))
        return NSGA3_EINVAL;
    const Layout L = make_layout(M, m, 1, M);
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    if (n_stop <= 0 || n_stop > M) n_stop = M;
    const Ptrs P = carve(L, ws);
    return to_status(launch_nd_sort(L, P, F, n_stop, rank, front_info, true, (hipStream_t)stream));
}

int nsga3_normalize(const float *F, const int32_t *rank, const int32_t *front_info, int32_t M,
                    int32_t m, float *Fn, float *ideal, double *intercept, int32_t *extreme,
                    int32_t *degenerate, void *ws, size_t ws_bytes, void *stream) {
    if (!F || !rank || !front_info || !Fn || !ideal || !intercept || !extreme || !degenerate ||
        !valid_shape(M, m, 1, 1) || !aligned(F, 4) || !aligned(Fn, 4) || !aligned(intercept, 8))
        return NSGA3_EINVAL;
    const Layout L = make_layout(M, m, 1, M);
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    const Ptrs P = carve(L, ws);
    return to_status(launch_normalize(L, P, F, rank, front_info, Fn, ideal, intercept, extreme,
                                      degenerate, true, (hipStream_t)stream));
}

int nsga3_associate(const float *Fn, const int32_t *rank, const int32_t *front_info, int32_t M,
                    int32_t m, const float *Z, int32_t H, int32_t *pi, float *dist, void *ws,
                    size_t ws_bytes, void *stream) {
    if (!Fn || !rank || !front_info || !Z || !pi || !dist || !valid_shape(M, m, H, 1) ||
        !aligned(Fn, 4) || !aligned(Z, 4))
        return NSGA3_EINVAL;
    const Layout L = make_layout(M, m, H, M);
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    const Ptrs P = carve(L, ws);
    return to_status(
        launch_associate(L, P, Fn, rank, front_info, Z, pi, dist, true, (hipStream_t)stream));
}

int nsga3_niche(const int32_t *rank, const int32_t *front_info, const int32_t *pi,
                const float *dist, int32_t M, int32_t H, int32_t N, uint64_t seed,
                int32_t *selected, void *ws, size_t ws_bytes, void *stream) {
    if (!rank || !front_info || !pi || !dist || !selected || !valid_shape(M, 2, H, N))
        return NSGA3_EINVAL;
    const Layout L = make_layout(M, 2, H, N);
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    const Ptrs P = carve(L, ws);
    return to_status(
        launch_niche(L, P, rank, front_info, pi, dist, seed, selected, true, (hipStream_t)stream));
}

int nsga3_select(const float *F, int32_t M, int32_t m, const float *Z, int32_t H, int32_t N,
                 uint64_t seed, int32_t *selected, int32_t *rank_out, int32_t *pi_out,
                 float *dist_out, void *ws, size_t ws_bytes, void *stream) {
    if (!F || !Z || !selected || !valid_shape(M, m, H, N) || !aligned(F, 4) || !aligned(Z, 4))
        return NSGA3_EINVAL;
    const Layout L = make_layout(M, m, H, N);
    int rc = check_ws(L, ws, ws_bytes);
    if (rc) return rc;
    const Ptrs P = carve(L, ws);
    hipStream_t s = (hipStream_t)stream;
    int *rank = rank_out ? rank_out : P.rank;
    int *pi = pi_out ? pi_out : P.pi;
    float *dist = dist_out ? dist_out : P.dist;
    int *fi = P.ctrl->front_info;
    hipError_t e = launch_nd_sort(L, P, F, N, rank, fi, true, s);
    if (e == hipSuccess)
        e = launch_normalize(L, P, F, rank, fi, P.fn, P.ctrl->ideal_out, P.ctrl->icpt_out,
                             P.ctrl->ext_out, &P.ctrl->degen_out, false, s);
    if (e == hipSuccess) e = launch_associate(L, P, P.fn, rank, fi, Z, pi, dist, false, s);
    if (e == hipSuccess) e = launch_niche(L, P, rank, fi, pi, dist, seed, selected, false, s);
    return to_status(e);
}

int nsga3_read_status(const void *ws, void *stream, int32_t *status) {
    if (!ws || !status) return NSGA3_EINVAL;
    int bits = 0;
    hipStream_t s = (hipStream_t)stream;
    const Ctrl *ctrl = (const Ctrl *)ws;
    if (hipMemcpyAsync(&bits, &ctrl->status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return NSGA3_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return NSGA3_EHIP;
    if (bits & ST_NONFINITE) *status = NSGA3_ENONFINITE;
    else if (bits & ST_BADREF) *status = NSGA3_EINVAL;
    else if (bits & ST_INTERNAL) *status = NSGA3_EINTERNAL;
    else *status = NSGA3_OK;
    return NSGA3_OK;
}

const char *nsga3_version(void) { return "nsga3-mi355x 0.1 (gfx950)"; }

int nsga3_profile_enable(const char *kernels) {
    g_prof.used = 0;
    g_prof.dropped = 0;
    if (!kernels || !kernels[0]) {
        g_prof.on = false;
        return NSGA3_OK;
    }
    if (strlen(kernels) >= sizeof(g_prof.filter)) return NSGA3_EINVAL;
    strcpy(g_prof.filter, kernels);
    g_prof.all = strcmp(kernels, "*") == 0;
    while (g_prof.created < PROF_POOL) {
        if (hipEventCreate(&g_prof.ev[2 * g_prof.created]) != hipSuccess) return NSGA3_EHIP;
        if (hipEventCreate(&g_prof.ev[2 * g_prof.created + 1]) != hipSuccess) {
            (void)hipEventDestroy(g_prof.ev[2 * g_prof.created]);
            return NSGA3_EHIP;
        }
        ++g_prof.created;
    }
    g_prof.on = true;
    return NSGA3_OK;
}

int nsga3_profile_read(const char *kernel, double *total_ms, int64_t *launches,
                       int32_t *dropped) {
    if (!kernel || !total_ms || !launches) return NSGA3_EINVAL;
    double tot = 0.0;
    int64_t n = 0;
    for (int i = 0; i < g_prof.used; ++i) {
        if (strcmp(g_prof.rec_name[i], kernel) != 0) continue;
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess) return NSGA3_EHIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess)
            return NSGA3_EHIP;
        tot += ms;
        ++n;
    }
    *total_ms = tot;
    *launches = n;
    if (dropped) *dropped = g_prof.dropped;
    return NSGA3_OK;
}

}  // extern "C"

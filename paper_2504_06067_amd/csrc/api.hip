// C-ABI entry points of libnsga3: host-side validation, workspace carving,
// the batch plan, and the ordered enqueue of each stage's kernels. No call
// allocates device memory or waits for the device, except the status reads
// (which wait by design).
//
// Workspace of a call with B instances: the instance regions one after the
// other (instance 0 at offset 0, so its control block, and the status word,
// sit at the start of the workspace), then the batch header (descriptors and
// prefix arrays), which the call's first kernels write from their arguments.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

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
    L.ctrl = take(sizeof(Ctrl));
    L.ft = take((size_t)m * Mp * 4);
    L.nd = take(Mp * 4);
    L.mask = take(W * Mp * 8);
    L.ring = take((size_t)PEEL_RING * front_slot_words(L.W) * 8);  // peel front ring
    L.perm = take(Mp * 4);
    L.pkey = take(Mp * 4);
    L.bcount = take((size_t)PLACE_BUCKETS * 4);
    L.row_ord = take(W * 4);
    L.col_end = take(W * 4);
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
    L.qrow = take(Mp * 4);
    L.picked = take(Mp * 4);
    L.tcnt = take((Mp + COMPACT_TILE - 1) / COMPACT_TILE * 4);
    L.remain = take((W + (size_t)H + 2) * 8);
    L.emat = take(m > NARROW_M ? ((size_t)m * m + 3 * (size_t)m) * 8 : 0);
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
    P.ring = (u64 *)(b + L.ring);
    P.perm = (int *)(b + L.perm);
    P.pkey = (unsigned *)(b + L.pkey);
    P.bcount = (unsigned *)(b + L.bcount);
    P.row_ord = (int *)(b + L.row_ord);
    P.col_end = (int *)(b + L.col_end);
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
    P.qrow = (int *)(b + L.qrow);
    P.picked = (int *)(b + L.picked);
    P.tcnt = (int *)(b + L.tcnt);
    P.remain = (u64 *)(b + L.remain);
    P.emat = (double *)(b + L.emat);
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

static int to_status(hipError_t e) { return e == hipSuccess ? NSGA3_OK : NSGA3_EHIP; }

// ------------------------------------------------------------ batch header

// Byte offsets inside the batch header.
struct HeaderLayout {
    size_t tab, pt_pref, ref_pref, chunk_pref, order, dom_pref, asc_pref, ticket, total;
};

static HeaderLayout header_layout(int B) {
    HeaderLayout h;
    size_t o = 0;
    auto take = [&o](size_t bytes) { size_t at = o; o += up256(bytes); return at; };
    h.tab = take((size_t)B * sizeof(Inst));
    h.pt_pref = take((size_t)(B + 1) * 4);
    h.ref_pref = take((size_t)(B + 1) * 4);
    h.chunk_pref = take((size_t)(B + 1) * 4);
    h.order = take((size_t)B * 4);
    h.dom_pref = take((size_t)(B + 1) * 8);
    h.asc_pref = take((size_t)(B + 1) * 8);
    h.ticket = take((size_t)TICKET_SHARDS * TICKET_STRIDE * 8);
    h.total = o;
    return h;
}

// Association slicing: references per slice so that the whole batch holds
// about ASSOC_WAVES waves (a lone large instance gets many slices, a large
// batch whole reference sets per wave).
constexpr long long ASSOC_WAVES = 16384;

// Dominance tiles per work item when the caller does not choose. A launch
// (the instances of equal m) is cut into about DOM_ROUNDS rounds of waves,
// DOM_WAVES_PER_CU per compute unit (4 SIMDs x 8 waves), with 1 to
// DOM_MAX_TILES tiles per item: measured on one MI355X, a single round of
// long items loses 10-25 % to uneven wave placement, and items of 2-3 tiles
// amortize the per-item setup (one tile per item costs up to 8 % on small
// triangles; two rounds give the large workload's 49 k tiles 3 tiles per
// item, 35.5 us against 36.0 us with three rounds of 2-tile items).
// Launches of millions of tiles take longer items: the waves
// of 3-tile items averaged 3.9 resident per SIMD of 7 (per-wave setup and
// the refill of finished workgroups), and 12 tiles per item cut the
// many-objective launch (2.1 M tiles) from 3.55 to 3.40 ms; 96 are slower.
constexpr long long DOM_WAVES_PER_CU = 32;
constexpr long long DOM_ROUNDS = 2;
constexpr long long DOM_MAX_TILES = 12;

static int auto_slice(int H, long long sum_W, int m) {
    long long R = (long long)H * sum_W / ASSOC_WAVES;
    R = ((R + 15) / 16) * 16;
    // a reference costs a wave about 3m operations: above NARROW_M the
    // slices stay short so that few points still spread over many waves
    const long long lo = m > NARROW_M ? 16 : 32;
    if (R < lo) R = lo;
    if (R > H) R = H;
    return (int)R;
}

// One instance's shape and caller pointers, before placement.
struct Spec {
    Inst I;     // caller pointers and shape; P filled by plan()
    int tile[4];
    char *own;  // the instance's own workspace region, or null
    size_t own_bytes;
};

// Copies 4-byte words of the batch header from the kernel arguments.
constexpr int BLOB_WORDS = 768;
struct Blob {
    unsigned w[BLOB_WORDS];
};

__global__ __launch_bounds__(256) void k_blob(Blob b, unsigned *dst, int n) {
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = b.w[i];
}

// The whole header of a one-instance call, and the start of that instance
// (as k_init), in one launch.
__global__ __launch_bounds__(256) void k_blob_init(Blob b, unsigned *dst, int n, Ctrl *ctrl,
                                                   int *front_info, int n_stop, int run,
                                                   unsigned *bcount, u64 *ticket) {
    for (int i = threadIdx.x; i < n; i += 256) dst[i] = b.w[i];
    init_instance(ctrl, front_info, n_stop, run, bcount, threadIdx.x);
    if (threadIdx.x < TICKET_SHARDS) ticket[threadIdx.x * TICKET_STRIDE] = 0;
}

// A planned call: per-instance regions, the header bytes, the host plan and
// the device view.
struct Plan {
    std::vector<Layout> lay;
    std::vector<size_t> region;   // offset in the call's workspace (own regions: unused)
    std::vector<char *> base;     // start of each instance's region
    size_t inst_total = 0;
    HeaderLayout hl;
    size_t total = 0;
    std::vector<unsigned char> hdr;
    HostPlan hp;
    BatchView bv;
};

static bool valid_tiles(const int *t, int H) {
    if (t[0] < 0 || t[0] > (1 << 30)) return false;
    if (t[1] < 0 || t[1] > H) return false;
    if (t[1] != 0 && t[1] != H && (t[1] < 16 || t[1] % 16 != 0)) return false;
    return t[2] == 0 && t[3] == 0;
}

// Sizes only (ws == nullptr) or sizes, header bytes and device view.
static void plan(std::vector<Spec> &spec, char *ws, int run, Plan &p) {
    const int B = (int)spec.size();
    p.lay.resize(B);
    p.region.resize(B);
    size_t o = 0;
    long long sum_W = 0;
    for (int b = 0; b < B; ++b) {
        const Inst &I = spec[b].I;
        p.lay[b] = make_layout(I.M, I.m, I.H, I.N);
        p.region[b] = o;
        if (!spec[b].own) o += p.lay[b].total;
        sum_W += p.lay[b].W;
    }
    p.inst_total = o;
    p.hl = header_layout(B);
    p.total = o + p.hl.total;
    if (!ws) return;
    p.base.resize(B);
    for (int b = 0; b < B; ++b) p.base[b] = spec[b].own ? spec[b].own : ws + p.region[b];

    std::vector<Inst> tab(B);
    std::vector<int> pt(B + 1), ref(B + 1), chunk(B + 1), order(B);
    std::vector<long long> dom(B + 1), asc(B + 1);
    pt[0] = ref[0] = chunk[0] = 0;
    for (int b = 0; b < B; ++b) {
        const Layout &L = p.lay[b];
        Inst I = spec[b].I;
        I.P = carve(L, p.base[b]);
        I.Mp = L.Mp;
        I.W = L.W;
        I.Hp = L.Hp;
        I.G = spec[b].tile[0];  // 0: set per launch group below
        I.R = spec[b].tile[1] > 0 ? spec[b].tile[1] : auto_slice(I.H, sum_W, I.m);
        I.nslice = (I.H + I.R - 1) / I.R;
        tab[b] = I;
        pt[b + 1] = pt[b] + (int)((I.M + PT_ALIGN - 1) / PT_ALIGN * PT_ALIGN);
        ref[b + 1] = ref[b] + (int)((I.Hp + PT_ALIGN - 1) / PT_ALIGN * PT_ALIGN);
        order[b] = b;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return tab[a].m < tab[c].m; });
    HostPlan &hp = p.hp;
    hp.B = B;
    hp.npt = pt[B];
    hp.nref = ref[B];
    hp.ngroups = 0;
    hp.max_W = 0;
    for (int i = 0; i < B; ++i) {
        const Inst &I = tab[order[i]];
        chunk[i + 1] = chunk[i] + I.W;
        if (I.W > hp.max_W) hp.max_W = I.W;
        if (i == 0 || I.m != tab[order[i - 1]].m) {
            hp.grp_m[hp.ngroups] = I.m;
            hp.grp_start[hp.ngroups] = i;
            hp.grp_chunk[hp.ngroups] = chunk[i];
            hp.grp_max_W[hp.ngroups] = 0;
            ++hp.ngroups;
        }
        int &gw = hp.grp_max_W[hp.ngroups - 1];
        if (I.W > gw) gw = I.W;
    }
    hp.nchunk = chunk[B];
    hp.grp_start[hp.ngroups] = B;
    hp.grp_chunk[hp.ngroups] = chunk[B];
    const long long dom_waves = DOM_WAVES_PER_CU * device_info().cus;
    for (int g = 0; g < hp.ngroups; ++g) {
        long long tiles = 0;
        for (int i = hp.grp_start[g]; i < hp.grp_start[g + 1]; ++i) tiles += dominance_tiles(tab[order[i]].W);
        const long long per = DOM_ROUNDS * dom_waves;
        long long G = (tiles + per / 2) / per;
        G = G < 1 ? 1 : (G > DOM_MAX_TILES ? DOM_MAX_TILES : G);
        for (int i = hp.grp_start[g]; i < hp.grp_start[g + 1]; ++i)
            if (tab[order[i]].G == 0) tab[order[i]].G = (int)G;
    }
    dom[0] = asc[0] = 0;
    for (int i = 0; i < B; ++i) {
        const Inst &I = tab[order[i]];
        dom[i + 1] = dom[i] + (dominance_tiles(I.W) + I.G - 1) / I.G;
        asc[i + 1] = asc[i] + (long long)I.W * I.nslice;
    }
    for (int g = 0; g <= hp.ngroups; ++g) {
        hp.grp_dom[g] = dom[hp.grp_start[g]];
        hp.grp_asc[g] = asc[hp.grp_start[g]];
    }

    // header bytes
    const HeaderLayout &hl = p.hl;
    // everything before the ticket counters (which k_init zeroes) is uploaded
    p.hdr.assign(hl.ticket, 0);
    unsigned char *h = p.hdr.data();
    memcpy(h + hl.tab, tab.data(), (size_t)B * sizeof(Inst));
    memcpy(h + hl.pt_pref, pt.data(), (size_t)(B + 1) * 4);
    memcpy(h + hl.ref_pref, ref.data(), (size_t)(B + 1) * 4);
    memcpy(h + hl.chunk_pref, chunk.data(), (size_t)(B + 1) * 4);
    memcpy(h + hl.order, order.data(), (size_t)B * 4);
    memcpy(h + hl.dom_pref, dom.data(), (size_t)(B + 1) * 8);
    memcpy(h + hl.asc_pref, asc.data(), (size_t)(B + 1) * 8);

    char *hd = ws + p.inst_total;
    BatchView &bv = p.bv;
    bv.tab = (CInst *)(hd + hl.tab);
    bv.pt_pref = (const NSGA3_RO int *)(hd + hl.pt_pref);
    bv.ref_pref = (const NSGA3_RO int *)(hd + hl.ref_pref);
    bv.chunk_pref = (const NSGA3_RO int *)(hd + hl.chunk_pref);
    bv.order = (const NSGA3_RO int *)(hd + hl.order);
    bv.dom_pref = (const NSGA3_RO long long *)(hd + hl.dom_pref);
    bv.asc_pref = (const NSGA3_RO long long *)(hd + hl.asc_pref);
    bv.ticket = (u64 *)(hd + hl.ticket);
    bv.B = B;
    bv.run = run;
}

hipError_t upload(const void *src_, size_t bytes, void *dst_, hipStream_t s) {
    unsigned *dst = (unsigned *)dst_;
    const unsigned *src = (const unsigned *)src_;
    const int words = (int)(bytes / 4);
    Blob blob;
    for (int w0 = 0; w0 < words; w0 += BLOB_WORDS) {
        const int n = std::min(BLOB_WORDS, words - w0);
        memcpy(blob.w, src + w0, (size_t)n * 4);
        NSGA3_LAUNCH("header", k_blob, dim3(1), dim3(256), 0, s, blob, dst + w0, n);
    }
    return hipGetLastError();
}

// Enqueues the header copy, then the stages of `run`.
static hipError_t enqueue(Plan &p, char *ws, hipStream_t s) {
    hipError_t e;
    const bool fused = p.hp.B == 1 && p.hdr.size() <= sizeof(Blob);
    if (fused) {
        Blob blob;
        memcpy(blob.w, p.hdr.data(), p.hdr.size());
        Inst I0;
        memcpy(&I0, p.hdr.data() + p.hl.tab, sizeof(Inst));
        NSGA3_LAUNCH("header", k_blob_init, dim3(1), dim3(256), 0, s, blob,
                     (unsigned *)(ws + p.inst_total), (int)(p.hdr.size() / 4), I0.P.ctrl,
                     I0.front_info, I0.n_stop, p.bv.run, I0.P.bcount, p.bv.ticket);
        e = hipGetLastError();
    } else {
        e = upload(p.hdr.data(), p.hdr.size(), ws + p.inst_total, s);
    }
    if (e == hipSuccess) e = launch_prepare(p.hp, p.bv, fused, s);
    const int run = p.bv.run;
    // a whole selection whose m-groups all take the one-pass normalization
    // may run each group's normalization and association sweep right after
    // its peel
    bool through = (run & RUN_ND) && (run & RUN_NORM) && (run & RUN_ASSOC);
    for (int g = 0; g < p.hp.ngroups && through; ++g) through = p.hp.grp_m[g] <= NARROW_M;
    if (e == hipSuccess && (run & RUN_ND)) e = launch_nd_sort(p.hp, p.bv, s, &through);
    else through = false;
    if (e == hipSuccess && (run & RUN_NORM) && !through) e = launch_normalize(p.hp, p.bv, s);
    if (e == hipSuccess && (run & RUN_ASSOC)) e = launch_associate(p.hp, p.bv, s, through);
    if (e == hipSuccess && (run & RUN_NICHE)) e = launch_niche(p.hp, p.bv, s);
    return e;
}

static Spec blank_spec(int M, int m, int H, int N) {
    Spec sp;
    memset(&sp, 0, sizeof(sp));
    sp.I.M = M;
    sp.I.m = m;
    sp.I.H = H;
    sp.I.N = N;
    sp.I.n_stop = N;
    return sp;
}

static int check_ws(size_t need, const void *ws, size_t ws_bytes) {
    if (!ws || !aligned(ws, 256)) return NSGA3_EINVAL;
    if (ws_bytes < need) return NSGA3_EWORKSPACE;
    return NSGA3_OK;
}

// Runs a one-instance call of the stages in `run`.
static int run_single(Spec sp, void *ws, size_t ws_bytes, int run, hipStream_t s) {
    std::vector<Spec> v(1, sp);
    Plan p;
    plan(v, nullptr, run, p);
    const int rc = check_ws(p.total, ws, ws_bytes);
    if (rc) return rc;
    plan(v, (char *)ws, run, p);
    return to_status(enqueue(p, (char *)ws, s));
}

static bool valid_instance(const nsga3_instance &q) {
    return q.F && q.Z && q.selected && valid_shape(q.M, q.m, q.H, q.N) && aligned(q.F, 4) &&
           aligned(q.Z, 4) && aligned(q.selected, 4) && (!q.rank || aligned(q.rank, 4)) &&
           (!q.pi || aligned(q.pi, 4)) && (!q.dist || aligned(q.dist, 4)) &&
           valid_tiles(q.tile, q.H);
}

static void specs_of(const nsga3_instance *inst, int B, std::vector<Spec> &v) {
    v.resize(B);
    for (int b = 0; b < B; ++b) {
        const nsga3_instance &q = inst[b];
        v[b] = blank_spec(q.M, q.m, q.H, q.N);
        v[b].I.F = q.F;
        v[b].I.Z = q.Z;
        v[b].I.selected = q.selected;
        v[b].I.rank = q.rank;
        v[b].I.pi = q.pi;
        v[b].I.dist = q.dist;
        v[b].I.seed = q.seed;
        for (int t = 0; t < 4; ++t) v[b].tile[t] = q.tile[t];
        v[b].own = (char *)q.ws;
        v[b].own_bytes = q.ws_bytes;
    }
}

// Internal destinations of a selection: rank/pi/dist default to the
// instance's region; front_info, Fn and the normalization outputs always do.
static void place_select(Plan &p, std::vector<Spec> &v, char *ws) {
    for (size_t b = 0; b < v.size(); ++b) {
        const Ptrs P = carve(p.lay[b], v[b].own ? v[b].own : ws + p.region[b]);
        Inst &I = v[b].I;
        if (!I.rank) I.rank = P.rank;
        if (!I.pi) I.pi = P.pi;
        if (!I.dist) I.dist = P.dist;
        I.front_info = P.ctrl->front_info;
        I.Fn = P.fn;
        I.ideal = P.ctrl->ideal_out;
        I.intercept = P.ctrl->icpt_out;
        I.extreme = P.ctrl->ext_out;
        I.degenerate = &P.ctrl->degen_out;
    }
}

static int run_select(std::vector<Spec> &v, void *ws, size_t ws_bytes, hipStream_t s) {
    Plan p;
    plan(v, nullptr, RUN_SELECT, p);
    int rc = check_ws(p.total, ws, ws_bytes);
    if (rc) return rc;
    for (size_t b = 0; b < v.size(); ++b)
        if (v[b].own && (rc = check_ws(p.lay[b].total, v[b].own, v[b].own_bytes))) return rc;
    place_select(p, v, (char *)ws);
    plan(v, (char *)ws, RUN_SELECT, p);
    return to_status(enqueue(p, (char *)ws, s));
}

// A one-instance selection small enough for one workgroup: the same plan
// and workspace (the status word and the internal outputs live where the
// multi-kernel path puts them), one launch.
static int run_select_tiny(std::vector<Spec> &v, void *ws, size_t ws_bytes, hipStream_t s) {
    Plan p;
    plan(v, nullptr, RUN_SELECT, p);
    const int rc = check_ws(p.total, ws, ws_bytes);
    if (rc) return rc;
    place_select(p, v, (char *)ws);
    plan(v, (char *)ws, RUN_SELECT, p);
    Inst I0;
    memcpy(&I0, p.hdr.data() + p.hl.tab, sizeof(Inst));
    return to_status(launch_select_tiny(I0, s));
}

static int run_select_one(std::vector<Spec> &v, void *ws, size_t ws_bytes, hipStream_t s) {
    const Inst &I = v[0].I;
    if (tiny_fits(I.M, I.m, I.H)) return run_select_tiny(v, ws, ws_bytes, s);
    return run_select(v, ws, ws_bytes, s);
}

static int status_code(int bits) {
    if (bits & ST_NONFINITE) return NSGA3_ENONFINITE;
    if (bits & ST_BADREF) return NSGA3_EINVAL;
    if (bits & ST_INTERNAL) return NSGA3_EINTERNAL;
    return NSGA3_OK;
}

// ------------------------------------------------------ no-alloc scratch

// The workspace of nsga3_select_noalloc: a device array of the library, one
// copy per GPU, held until the process ends. Host code never passes `scratch`
// itself to a kernel (in host code it names a host-side stand-in); it uses
// the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[NSGA3_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch[MAX_DEVICES];
}  // namespace

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
static hipError_t scratch_of_current_device(char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr || !aligned(ptr, 256)) return hipErrorInvalidSymbol;
        g_scratch[dev] = (char *)ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// The public status code of an instance, from its control block.
__global__ void k_status_out(const Ctrl *ctrl, int *status) {
    if (threadIdx.x != 0) return;
    const int bits = ctrl->status;
    *status = (bits & ST_NONFINITE)  ? NSGA3_ENONFINITE
              : (bits & ST_BADREF)   ? NSGA3_EINVAL
              : (bits & ST_INTERNAL) ? NSGA3_EINTERNAL
                                     : NSGA3_OK;
}

// ---------------------------------------------------------- instrumentation

namespace {
constexpr int PROF_POOL = 8192;   // event pairs per enable
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
    std::vector<Spec> v(1, blank_spec(M, m, H, N));
    Plan p;
    plan(v, nullptr, RUN_SELECT, p);
    return p.total;
}

int nsga3_nd_sort(const float *F, int32_t M, int32_t m, int32_t n_stop, int32_t *rank,
                  int32_t *front_info, void *ws, size_t ws_bytes, void *stream) {
    if (!F || !rank || !front_info || !valid_shape(M, m, 1, 1) || !aligned(F, 4) ||
        !aligned(rank, 4) || !aligned(front_info, 4))
        return NSGA3_EINVAL;
    if (n_stop <= 0 || n_stop > M) n_stop = M;
    Spec sp = blank_spec(M, m, 1, M);
    sp.I.F = F;
    sp.I.rank = rank;
    sp.I.front_info = front_info;
    sp.I.n_stop = n_stop;
    return run_single(sp, ws, ws_bytes, RUN_ND, (hipStream_t)stream);
}

int nsga3_normalize(const float *F, const int32_t *rank, const int32_t *front_info, int32_t M,
                    int32_t m, float *Fn, float *ideal, double *intercept, int32_t *extreme,
                    int32_t *degenerate, void *ws, size_t ws_bytes, void *stream) {
    if (!F || !rank || !front_info || !Fn || !ideal || !intercept || !extreme || !degenerate ||
        !valid_shape(M, m, 1, 1) || !aligned(F, 4) || !aligned(Fn, 4) || !aligned(intercept, 8))
        return NSGA3_EINVAL;
    Spec sp = blank_spec(M, m, 1, M);
    sp.I.F = F;
    sp.I.rank = (int *)rank;              // read only in this call
    sp.I.front_info = (int *)front_info;  // read only in this call
    sp.I.Fn = Fn;
    sp.I.ideal = ideal;
    sp.I.intercept = intercept;
    sp.I.extreme = extreme;
    sp.I.degenerate = degenerate;
    return run_single(sp, ws, ws_bytes, RUN_NORM, (hipStream_t)stream);
}

int nsga3_associate(const float *Fn, const int32_t *rank, const int32_t *front_info, int32_t M,
                    int32_t m, const float *Z, int32_t H, int32_t *pi, float *dist, void *ws,
                    size_t ws_bytes, void *stream) {
    if (!Fn || !rank || !front_info || !Z || !pi || !dist || !valid_shape(M, m, H, 1) ||
        !aligned(Fn, 4) || !aligned(Z, 4))
        return NSGA3_EINVAL;
    Spec sp = blank_spec(M, m, H, M);
    sp.I.Fn = (float *)Fn;                // read only in this call
    sp.I.rank = (int *)rank;
    sp.I.front_info = (int *)front_info;
    sp.I.Z = Z;
    sp.I.pi = pi;
    sp.I.dist = dist;
    return run_single(sp, ws, ws_bytes, RUN_ASSOC, (hipStream_t)stream);
}

int nsga3_niche(const int32_t *rank, const int32_t *front_info, const int32_t *pi,
                const float *dist, int32_t M, int32_t H, int32_t N, uint64_t seed,
                int32_t *selected, void *ws, size_t ws_bytes, void *stream) {
    if (!rank || !front_info || !pi || !dist || !selected || !valid_shape(M, 2, H, N))
        return NSGA3_EINVAL;
    Spec sp = blank_spec(M, 2, H, N);
    sp.I.rank = (int *)rank;              // read only in this call
    sp.I.front_info = (int *)front_info;
    sp.I.pi = (int *)pi;
    sp.I.dist = (float *)dist;
    sp.I.seed = seed;
    sp.I.selected = selected;
    return run_single(sp, ws, ws_bytes, RUN_NICHE, (hipStream_t)stream);
}

int nsga3_niche_cache_tensor(const int32_t *rank, const int32_t *front_info, const int32_t *pi,
                             const float *dist, int32_t M, int32_t H, int32_t N, uint64_t seed,
                             int32_t *selected, void *ws, size_t ws_bytes, void *stream) {
    if (!rank || !front_info || !pi || !dist || !selected || !valid_shape(M, 2, H, N))
        return NSGA3_EINVAL;
    Spec sp = blank_spec(M, 2, H, N);
    sp.I.rank = (int *)rank;              // read only in this call
    sp.I.front_info = (int *)front_info;
    sp.I.pi = (int *)pi;
    sp.I.dist = (float *)dist;
    sp.I.seed = seed;
    sp.I.selected = selected;
    return run_single(sp, ws, ws_bytes, RUN_NICHE | RUN_CACHE_TENSOR, (hipStream_t)stream);
}

int nsga3_select(const float *F, int32_t M, int32_t m, const float *Z, int32_t H, int32_t N,
                 uint64_t seed, int32_t *selected, int32_t *rank_out, int32_t *pi_out,
                 float *dist_out, void *ws, size_t ws_bytes, void *stream) {
    nsga3_instance q;
    memset(&q, 0, sizeof(q));
    q.F = F;
    q.Z = Z;
    q.selected = selected;
    q.rank = rank_out;
    q.pi = pi_out;
    q.dist = dist_out;
    q.M = M;
    q.m = m;
    q.H = H;
    q.N = N;
    q.seed = seed;
    if (!valid_instance(q)) return NSGA3_EINVAL;
    std::vector<Spec> v;
    specs_of(&q, 1, v);
    return run_select_one(v, ws, ws_bytes, (hipStream_t)stream);
}

int nsga3_select_noalloc(const float *F, int32_t M, int32_t m, const float *Z, int32_t H,
                         int32_t N, uint64_t seed, int32_t *selected, int32_t *rank_out,
                         int32_t *pi_out, float *dist_out, int32_t *status, void *stream) {
    nsga3_instance q;
    memset(&q, 0, sizeof(q));
    q.F = F;
    q.Z = Z;
    q.selected = selected;
    q.rank = rank_out;
    q.pi = pi_out;
    q.dist = dist_out;
    q.M = M;
    q.m = m;
    q.H = H;
    q.N = N;
    q.seed = seed;
    if (!valid_instance(q) || (status && !aligned(status, 4))) return NSGA3_EINVAL;
    std::vector<Spec> v;
    specs_of(&q, 1, v);
    {
        Plan p;
        plan(v, nullptr, RUN_SELECT, p);
        if (p.total > NSGA3_NOALLOC_SCRATCH_BYTES) return NSGA3_EWORKSPACE;
    }
    char *ws = nullptr;
    if (scratch_of_current_device(&ws) != hipSuccess) return NSGA3_EHIP;
    hipStream_t s = (hipStream_t)stream;
    const int rc = run_select_one(v, ws, NSGA3_NOALLOC_SCRATCH_BYTES, s);
    if (rc != NSGA3_OK || !status) return rc;
    // instance 0's control block sits at the start of the scratch
    NSGA3_LAUNCH("status", k_status_out, dim3(1), dim3(64), 0, s, (const Ctrl *)ws, status);
    return to_status(hipGetLastError());
}

size_t nsga3_instance_workspace_bytes(int32_t M, int32_t m, int32_t H, int32_t N) {
    if (!valid_shape(M, m, H, N)) return 0;
    return make_layout(M, m, H, N).total;
}

size_t nsga3_evolve_workspace_bytes(int32_t B) {
    if (B < 1 || B > NSGA3_MAX_BATCH) return 0;
    return evolve_header_bytes(B);
}

int nsga3_evolve_batched(const nsga3_evolve_slot *slots, int32_t B, void *ws, size_t ws_bytes,
                         void *stream) {
    if (!slots || B < 1 || B > NSGA3_MAX_BATCH) return NSGA3_EINVAL;
    for (int b = 0; b < B; ++b) {
        const nsga3_evolve_slot &q = slots[b];
        const bool needs_old = q.mode != NSGA3_EVOLVE_INIT;
        if (q.mode < NSGA3_EVOLVE_GENERATION || q.mode > NSGA3_EVOLVE_INIT || q.reserved != 0 ||
            q.N < 1 || q.N > NSGA3_MAX_POINTS / 2 || q.d < 2 || q.d > NSGA3_MAX_DECISION ||
            q.m < 2 || q.m > NSGA3_MAX_EVOLVE_OBJECTIVES || q.generation < 0 ||
            q.generation > 65535 || !q.X_new || !q.F_new || !q.A ||
            (needs_old && (!q.X_old || !q.F_old)) || !aligned(q.X_new, 4) ||
            !aligned(q.F_new, 4) || !aligned(q.A, 4))
            return NSGA3_EINVAL;
    }
    const int rc = check_ws(evolve_header_bytes(B), ws, ws_bytes);
    if (rc) return rc;
    return to_status(launch_evolve(slots, B, (char *)ws, (hipStream_t)stream));
}

size_t nsga3_batched_workspace_bytes(const nsga3_instance *inst, int32_t B) {
    if (!inst || B < 1 || B > NSGA3_MAX_BATCH) return 0;
    for (int b = 0; b < B; ++b)
        if (!valid_shape(inst[b].M, inst[b].m, inst[b].H, inst[b].N) ||
            !valid_tiles(inst[b].tile, inst[b].H))
            return 0;
    std::vector<Spec> v;
    specs_of(inst, B, v);
    Plan p;
    plan(v, nullptr, RUN_SELECT, p);
    return p.total;
}

int nsga3_select_batched(const nsga3_instance *inst, int32_t B, void *ws, size_t ws_bytes,
                         void *stream) {
    if (!inst || B < 1 || B > NSGA3_MAX_BATCH) return NSGA3_EINVAL;
    for (int b = 0; b < B; ++b)
        if (!valid_instance(inst[b])) return NSGA3_EINVAL;
    std::vector<Spec> v;
    specs_of(inst, B, v);
    return run_select(v, ws, ws_bytes, (hipStream_t)stream);
}

int nsga3_read_status(const void *ws, void *stream, int32_t *status) {
    if (!ws || !status) return NSGA3_EINVAL;
    int bits = 0;
    hipStream_t s = (hipStream_t)stream;
    const Ctrl *ctrl = (const Ctrl *)ws;
    if (hipMemcpyAsync(&bits, &ctrl->status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess)
        return NSGA3_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return NSGA3_EHIP;
    *status = status_code(bits);
    return NSGA3_OK;
}

int nsga3_read_status_batched(const nsga3_instance *inst, int32_t B, const void *ws,
                              void *stream, int32_t *status) {
    if (!inst || !ws || !status || B < 1 || B > NSGA3_MAX_BATCH) return NSGA3_EINVAL;
    for (int b = 0; b < B; ++b)
        if (!valid_shape(inst[b].M, inst[b].m, inst[b].H, inst[b].N)) return NSGA3_EINVAL;
    std::vector<Spec> v;
    specs_of(inst, B, v);
    Plan p;
    plan(v, nullptr, RUN_SELECT, p);
    hipStream_t s = (hipStream_t)stream;
    std::vector<int> bits(B, 0);
    for (int b = 0; b < B; ++b) {
        const char *base = inst[b].ws ? (const char *)inst[b].ws : (const char *)ws + p.region[b];
        const Ctrl *ctrl = (const Ctrl *)base;
        if (hipMemcpyAsync(&bits[b], &ctrl->status, sizeof(int), hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return NSGA3_EHIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return NSGA3_EHIP;
    for (int b = 0; b < B; ++b) status[b] = status_code(bits[b]);
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

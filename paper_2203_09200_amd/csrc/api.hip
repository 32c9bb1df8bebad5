// C ABI of librfsr: argument validation, workspace layout, job construction
// and stage sequencing.  Every step of the reconstruction runs in the kernels
// of fsr.hip and motion.hip; this file only validates, carves the caller's
// workspace, builds the jobs the kernels read and enqueues launches on the
// caller's stream.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.h"

using namespace rfsr;

namespace {

constexpr int32_t kVersion = 10800;   // 1.8.0
constexpr int kMaxBatch = 4096;

rfsr_status from_hip(hipError_t e) { return e == hipSuccess ? RFSR_OK : RFSR_EDEVICE; }

rfsr_status check_shape(int32_t H, int32_t W, int64_t pitch) {
    if (H <= 0 || W <= 0 || H > kMaxDim || W > kMaxDim) return RFSR_ESHAPE;
    if (H % kBlock != 0 || W % kBlock != 0) return RFSR_ESHAPE;
    if (pitch < W || pitch > (int64_t)1 << 30) return RFSR_ESHAPE;
    return RFSR_OK;
}

rfsr_status check_me(const rfsr_me_params* me) {
    if (!me) return RFSR_EINVAL;
    if (me->tmpl < 1 || me->tmpl > 8) return RFSR_EINVAL;
    if (me->search < 0 || me->search > kMaxSearch) return RFSR_EINVAL;
    if (me->check < RFSR_CHECK_NONE || me->check > RFSR_CHECK_NNC_FRMC) return RFSR_EINVAL;
    if (me->rmc_radius < 0 || me->rmc_radius > kMaxSearch) return RFSR_EINVAL;
    if (me->cost_norm != 0 && me->cost_norm != 1) return RFSR_EINVAL;
    if (me->nnc_center != RFSR_NNC_FILTERED && me->nnc_center != RFSR_NNC_RAW) return RFSR_EINVAL;
    if (me->n_frmc < 0 || me->n_frmc > kMaxFrmc) return RFSR_EINVAL;
    if (me->n_frmc > 0) {   // strictly increasing, containing 0, inside the window plane's reach
        bool zero = false;
        for (int i = 0; i < me->n_frmc; ++i) {
            const int d = me->frmc[i];
            if (d < -kMaxFrmcOffset || d > kMaxFrmcOffset) return RFSR_EINVAL;
            if (i > 0 && d <= me->frmc[i - 1]) return RFSR_EINVAL;
            zero |= d == 0;
        }
        if (!zero) return RFSR_EINVAL;
    }
    if (me->tmpl != 4) return RFSR_EUNSUPPORTED;
    return RFSR_OK;
}

rfsr_status check_fsr(const rfsr_fsr_params* p) {
    if (!p) return RFSR_EINVAL;
    if (p->iters < 0 || p->iters > kMaxIters) return RFSR_EINVAL;
    if (!(p->rho > 0.0 && p->rho <= 1.0)) return RFSR_EINVAL;
    if (!(p->gamma > 0.0 && p->gamma < 2.0)) return RFSR_EINVAL;
    if (!(p->proj_weight >= 0.0) || !isfinite(p->proj_weight)) return RFSR_EINVAL;
    if (p->overwrite != RFSR_DFSR && p->overwrite != RFSR_RFSR) return RFSR_EINVAL;
    if (p->block < 1 || p->support < p->block) return RFSR_EINVAL;
    if (p->precision < RFSR_PREC_FP64 || p->precision > RFSR_PREC_MIXED) return RFSR_EINVAL;
    if (p->precision == RFSR_PREC_MIXED && !(p->mixed_bound > 0.0 && p->mixed_bound <= 1e6)) return RFSR_EINVAL;
    if (!(p->concealed_weight >= 0.0 && p->concealed_weight <= 1.0)) return RFSR_EINVAL;
    if (p->pairs != 0 && p->pairs != 1) return RFSR_EINVAL;
    if (!(p->prior_sigma >= 0.0 && p->prior_sigma <= 1.0)) return RFSR_EINVAL;
    if (!(p->stop_ratio >= 0.0 && p->stop_ratio < 1.0)) return RFSR_EINVAL;
    if (p->pairs && p->concealed_weight > 0.0) return RFSR_EUNSUPPORTED;
    const bool f32 = p->precision == RFSR_PREC_FP32 || p->precision == RFSR_PREC_MIXED;
    if (f32 && (p->pairs || p->concealed_weight > 0.0)) return RFSR_EUNSUPPORTED;
    if ((p->prior_sigma > 0.0 || p->stop_ratio > 0.0) &&
        (p->pairs || p->concealed_weight > 0.0 || p->precision != RFSR_PREC_FP64))
        return RFSR_EUNSUPPORTED;
    if (p->block != kBlock || p->support != kSupport) return RFSR_EUNSUPPORTED;
    return RFSR_OK;
}

rfsr_status check_ws(void* ws, size_t have, size_t need) {
    if (!ws || ((uintptr_t)ws & 255u) != 0 || have < need) return RFSR_EWORKSPACE;
    return RFSR_OK;
}

// Scratch of one frame, as offsets from the frame's base (planes of pitch W):
// n map, window plane, FSR input, and per reference the vectors, decisions,
// best forward cost, medians and reverse field.
struct FrameScratch {
    size_t nmap, fm, values, cls;
    size_t mv_a[3], mv_b[3], acc[3], cost[3], ma[3], mb[3], ra[3], rb[3];
    size_t bytes;
    FrameScratch(int H, int W, int nref) {
        const size_t px = (size_t)H * W;
        size_t o = 0;
        nmap = o; o = align256(o + px);
        fm = o; o = align256(o + sizeof(uint2) * (size_t)(H + 2 * kPad) * (W + 2 * kPad));
        values = o; o = align256(o + 4 * px);
        cls = o; o = align256(o + px);
        for (int k = 0; k < 3; ++k) {
            const size_t n = k < nref ? px : 0;
            mv_a[k] = o; o = align256(o + n);
            mv_b[k] = o; o = align256(o + n);
            acc[k] = o; o = align256(o + n);
            cost[k] = o; o = align256(o + 2 * n);
            ma[k] = o; o = align256(o + n);
            mb[k] = o; o = align256(o + n);
            ra[k] = o; o = align256(o + n);
            rb[k] = o; o = align256(o + n);
        }
        bytes = o;
    }
};

// Workspace of the single-frame entry points: FSR tables | the mixed form's
// recomputation list | frame scratch.
size_t single_ws(int H, int W, int nref) {
    return align256(sizeof(FsrTables)) + rerun_bytes((size_t)(H / kBlock) * (W / kBlock)) +
           FrameScratch(H, W, nref).bytes;
}

// One frame to reconstruct; rfsr_frame_desc and the single-frame arguments
// both become one of these.
struct Frame {
    const uint8_t* cur;
    const uint8_t* cur_mask;
    const uint8_t* ref_recon[3];
    const uint8_t* ref_meas[3];
    const uint8_t* ref_mask[3];
    float* out;
    uint8_t* out_u8;
    int nref, H, W;
    int64_t pitch;
};

rfsr_status check_frame(const Frame& f, bool need_out = true) {
    if (!f.cur || !f.cur_mask || (need_out && !f.out)) return RFSR_EINVAL;
    if (f.nref < 0 || f.nref > 3) return RFSR_EINVAL;
    for (int k = 0; k < f.nref; ++k)
        if (!f.ref_recon[k] || !f.ref_meas[k] || !f.ref_mask[k]) return RFSR_EINVAL;
    return check_shape(f.H, f.W, f.pitch);
}

// The frame job and the nref reference jobs of `f`, whose scratch starts at
// `base`.  The reverse tests of the frame path run only on projectable pixels
// (ref_mask set).  First-workgroup offsets are left at 0.
void make_jobs(const Frame& f, uint8_t* base, bool windows, FrameJob& fj, RefJob* rj) {
    const FrameScratch L(f.H, f.W, f.nref);
    memset(&fj, 0, sizeof(fj));
    fj.cur = f.cur;
    fj.cur_mask = f.cur_mask;
    fj.fm = windows ? reinterpret_cast<uint2*>(base + L.fm) : nullptr;
    fj.values = reinterpret_cast<float*>(base + L.values);
    fj.cls = base + L.cls;
    fj.out = f.out;
    fj.out_u8 = f.out_u8;
    fj.pitch = f.pitch;
    fj.opitch = f.W;
    fj.vpitch = f.W;
    fj.H = f.H;
    fj.W = f.W;
    fj.nref = f.nref;
    for (int k = 0; k < f.nref; ++k) {
        RefJob& j = rj[k];
        memset(&j, 0, sizeof(j));
        j.cur = f.cur;
        j.cur_mask = f.cur_mask;
        j.ref = f.ref_recon[k];
        j.ref_mask = f.ref_mask[k];
        j.mv_a = reinterpret_cast<int8_t*>(base + L.mv_a[k]);
        j.mv_b = reinterpret_cast<int8_t*>(base + L.mv_b[k]);
        j.accept = base + L.acc[k];
        j.cost = reinterpret_cast<uint16_t*>(base + L.cost[k]);
        j.nmap_w = k == 0 ? base + L.nmap : nullptr;   // n depends on the frame only (see plan_batch)
        j.nmap = base + L.nmap;
        j.fm = reinterpret_cast<const uint2*>(base + L.fm);
        j.ma = reinterpret_cast<int8_t*>(base + L.ma[k]);
        j.mb = reinterpret_cast<int8_t*>(base + L.mb[k]);
        j.ra = reinterpret_cast<int8_t*>(base + L.ra[k]);
        j.rb = reinterpret_cast<int8_t*>(base + L.rb[k]);
        j.pitch = f.pitch;
        j.opitch = f.W;
        j.cpitch = f.W;
        j.H = f.H;
        j.W = f.W;
        fj.mv_a[k] = j.mv_a;
        fj.mv_b[k] = j.mv_b;
        fj.accept[k] = j.accept;
        fj.ref_meas[k] = f.ref_meas[k];
        fj.ref_mask[k] = f.ref_mask[k];
    }
}

template <class J>
Jobs<J> single(const J& j) {
    Jobs<J> js;
    js.table = nullptr;
    js.n = 0;
    js.one = j;
    return js;
}

template <class J>
Jobs<J> table(const uint8_t* image, size_t offset, int n, unsigned long long key) {
    Jobs<J> js;
    memset(&js, 0, sizeof(js));
    js.table = reinterpret_cast<const J*>(image + offset);
    js.stamp = reinterpret_cast<const unsigned long long*>(image);
    js.key = key;
    js.n = n;
    return js;
}

// ------------------------------------------------------------------ batch --
Frame to_frame(const rfsr_frame_desc& d) {
    Frame f;
    f.cur = d.cur;
    f.cur_mask = d.cur_mask;
    for (int k = 0; k < 3; ++k) {
        f.ref_recon[k] = d.ref_recon[k];
        f.ref_meas[k] = d.ref_meas[k];
        f.ref_mask[k] = d.ref_mask[k];
    }
    f.out = d.out;
    f.out_u8 = d.out_u8;
    f.nref = d.nref;
    f.H = d.H;
    f.W = d.W;
    f.pitch = d.pitch;
    return f;
}

rfsr_status check_batch(const rfsr_frame_desc* d, int n) {
    if (!d || n <= 0 || n > kMaxBatch) return RFSR_EINVAL;
    for (int i = 0; i < n; ++i) {
        const rfsr_status st = check_frame(to_frame(d[i]));
        if (st != RFSR_OK) return st;
    }
    return RFSR_OK;
}

// Workspace of a batch: FSR tables | the mixed form's recomputation list
// (every block of the batch) | scratch of frame 0 | frame 1 | ...
// Job-table image: header | FrameJob[n] | RefJob[total references].
struct BatchLayout {
    int nrefs = 0;
    size_t table_bytes, refs_offset, total;
    std::vector<size_t> frame_base;
    BatchLayout(const rfsr_frame_desc* d, int n) : frame_base(n) {
        size_t blocks = 0;
        for (int i = 0; i < n; ++i) {
            nrefs += d[i].nref;
            blocks += (size_t)(d[i].H / kBlock) * (d[i].W / kBlock);
        }
        refs_offset = kTableHeader + sizeof(FrameJob) * (size_t)n;
        table_bytes = align256(refs_offset + sizeof(RefJob) * (size_t)nrefs);
        size_t o = align256(sizeof(FsrTables)) + rerun_bytes(blocks);
        for (int i = 0; i < n; ++i) {
            frame_base[i] = o;
            o += FrameScratch(d[i].H, d[i].W, d[i].nref).bytes;
        }
        total = o;
    }
};

// The share of the work that one call runs.  Whole frames (`all`): every
// reference, window planes, FSR tables, projection and FSR.  A frame split
// for pipelining at reference index `first`: the early part runs the motion
// path of references first..nref-1 and the window planes of the frames that
// have such references; the finish runs references 0..first-1, the window
// planes of the frames without early references, the tables, projection
// and FSR.
struct Part {
    enum Kind { ALL = 0, MOTION = 1, FINISH = 2 };
    int kind = ALL;
    int first = 0;
    bool finish() const { return kind != MOTION; }
    int r0() const { return kind == MOTION ? first : 0; }
    int r1(int nref) const { return kind == FINISH ? min(first, nref) : nref; }
    // window planes of a frame with nref references (if the check needs them)
    bool windows(int nref) const {
        return kind == ALL || (kind == MOTION ? nref > first : nref <= first);
    }
    static Part motion(int first) {
        Part p;
        p.kind = MOTION;
        p.first = first;
        return p;
    }
    static Part finish_from(int first) {
        Part p;
        p.kind = FINISH;
        p.first = first;
        return p;
    }
};

// FNV-1a over the descriptors, the check, the workspace address and the
// share of work: the table image is valid exactly for this combination.
unsigned long long batch_key(const rfsr_frame_desc* d, int n, int check, const void* ws,
                             const Part& part = Part()) {
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&h](const void* p, size_t len) {
        const uint8_t* b = static_cast<const uint8_t*>(p);
        for (size_t i = 0; i < len; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    const uintptr_t addr = reinterpret_cast<uintptr_t>(ws);
    const int pw[2] = {part.kind, part.first};
    mix(&n, sizeof(n));
    mix(&check, sizeof(check));
    mix(&addr, sizeof(addr));
    mix(pw, sizeof(pw));
    for (int i = 0; i < n; ++i) {
        // hash the fields, not the struct bytes (reserved / padding ignored)
        mix(&d[i].cur, sizeof(d[i].cur));
        mix(&d[i].cur_mask, sizeof(d[i].cur_mask));
        for (int k = 0; k < 3; ++k) {
            const bool used = k < d[i].nref;
            const void* p3[3] = {used ? d[i].ref_recon[k] : nullptr, used ? d[i].ref_meas[k] : nullptr,
                                 used ? d[i].ref_mask[k] : nullptr};
            mix(p3, sizeof(p3));
        }
        mix(&d[i].out, sizeof(d[i].out));
        mix(&d[i].out_u8, sizeof(d[i].out_u8));
        mix(&d[i].nref, sizeof(d[i].nref));
        mix(&d[i].H, sizeof(d[i].H));
        mix(&d[i].W, sizeof(d[i].W));
        mix(&d[i].pitch, sizeof(d[i].pitch));
    }
    return h;
}

// Jobs of a batch with their first-workgroup offsets in the merged grids.
struct BatchPlan {
    std::vector<FrameJob> frames;
    std::vector<RefJob> refs;
    int win = 0, tiles = 0, px_refs = 0, frmc = 0, px_frames = 0, blocks = 0;
};

BatchPlan plan_batch(const rfsr_frame_desc* d, int n, const rfsr_me_params& me, uint8_t* ws,
                     const BatchLayout& L, const Part& part = Part()) {
    BatchPlan p;
    p.frames.resize(n);
    p.refs.reserve(L.nrefs);
    for (int i = 0; i < n; ++i) {
        const Frame f = to_frame(d[i]);
        const bool windows = f.nref > 0 && check_needs_windows(me.check);
        RefJob rj[3];
        FrameJob& fj = p.frames[i];
        make_jobs(f, ws + L.frame_base[i], windows, fj, rj);
        fj.g_px = p.px_frames;
        fj.g_win = p.win;
        fj.g_blk = p.blocks;
        p.px_frames += px_groups(f.H, f.W);
        p.win += windows && part.windows(f.nref) ? win_groups(f.H, f.W) : 0;
        p.blocks += (f.H / kBlock) * (f.W / kBlock);
        const int k0 = part.r0();
        for (int k = k0; k < part.r1(f.nref); ++k) {
            // the n map depends on the frame only: the first reference a call
            // runs writes it (a frame split for pipelining writes it twice,
            // with the same values, the second time after the first call)
            rj[k].nmap_w = k == k0 ? const_cast<uint8_t*>(rj[k].nmap) : nullptr;
            rj[k].g_tile = p.tiles;
            rj[k].g_px = p.px_refs;
            rj[k].g_frmc = p.frmc;
            p.tiles += me_tiles(f.H, f.W);
            p.px_refs += px_groups(f.H, f.W);
            p.frmc += frmc_groups(f.H, f.W);
            p.refs.push_back(rj[k]);
        }
    }
    return p;
}

// Host image of a batch's job tables: header (with the batch key) |
// FrameJob[n] | RefJob[total references].
void write_image(const rfsr_frame_desc* frames, int n, const rfsr_me_params& me, uint8_t* ws,
                 const BatchLayout& L, uint8_t* img, const Part& part = Part()) {
    const BatchPlan p = plan_batch(frames, n, me, ws, L, part);
    memset(img, 0, L.table_bytes);
    TableHeader hdr;
    memset(&hdr, 0, sizeof(hdr));
    hdr.key = batch_key(frames, n, me.check, ws, part);
    hdr.n_frames = n;
    hdr.n_refs = (int)p.refs.size();
    memcpy(img, &hdr, sizeof(hdr));
    memcpy(img + kTableHeader, p.frames.data(), sizeof(FrameJob) * p.frames.size());
    if (!p.refs.empty()) memcpy(img + L.refs_offset, p.refs.data(), sizeof(RefJob) * p.refs.size());
}

// Job-table image of one frame with up to three references, small enough to
// travel as a kernel argument.
constexpr size_t kFrameTable = 1024;
static_assert(kTableHeader + sizeof(FrameJob) + 3 * sizeof(RefJob) <= kFrameTable, "frame job table");
struct FrameTableImage {
    uint32_t w[kFrameTable / 4];
};

// Writes a frame's job-table image into its workspace, in stream order and
// without a copy: one workgroup, one dword per thread.
__global__ __launch_bounds__(256) void write_table_kernel(FrameTableImage img, uint32_t* __restrict__ dst) {
    dst[threadIdx.x] = img.w[threadIdx.x];
}

// The launch chain of a batch whose job-table image is at `img` on the
// device: tables, window planes, forward ME and checks over all (frame,
// reference) pairs, projection, FSR; stage events around the stages.  With
// `upload`, that image is first written to `img` (after the start event).
hipError_t run_batch(const rfsr_frame_desc* frames, int n, const rfsr_me_params& me,
                     const rfsr_fsr_params* fsr, const uint8_t* img, const FrameTableImage* upload,
                     void* const* stage_events, uint8_t* ws, const BatchLayout& L, hipStream_t s,
                     const Part& part = Part()) {
    const BatchPlan p = plan_batch(frames, n, me, ws, L, part);   // grid sizes
    const unsigned long long key = batch_key(frames, n, me.check, ws, part);
    const Jobs<FrameJob> jf = table<FrameJob>(img, kTableHeader, n, key);
    const Jobs<RefJob> jr = table<RefJob>(img, L.refs_offset, (int)p.refs.size(), key);
    FsrTables* tab = reinterpret_cast<FsrTables*>(ws);
    unsigned* rerun = reinterpret_cast<unsigned*>(ws + align256(sizeof(FsrTables)));
    hipError_t e = hipSuccess;
    auto record = [&](int k) {
        if (stage_events && e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(stage_events[k]), s);
    };
    record(0);
    if (e == hipSuccess && upload) {
        hipLaunchKernelGGL(write_table_kernel, dim3(1), dim3(256), 0, s, *upload,
                           reinterpret_cast<uint32_t*>(const_cast<uint8_t*>(img)));
        e = hipGetLastError();
    }
    if (e == hipSuccess && part.finish()) e = launch_fsr_tables(tab, fsr->rho, fsr->prior_sigma, s, rerun);
    if (e == hipSuccess && !p.refs.empty()) {
        e = launch_windows(jf, p.win, s);
        if (e == hipSuccess) e = launch_motion(jr, p.tiles, p.px_refs, p.frmc, me, nullptr, s);
    }
    record(1);
    if (e == hipSuccess && part.finish()) e = launch_project(jf, p.px_frames, s);
    record(2);
    if (e == hipSuccess && part.finish()) e = launch_fsr(jf, p.blocks, *fsr, tab, s, p.frames.data(), rerun);
    record(3);
    return e;
}

// One frame's share of work (`part`) as a batch of one: validation, then the
// job-table image written into table slot `slot` after the frame's scratch
// (in stream order, by a one-workgroup kernel), then the launch chain.
rfsr_status frame_call(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                       const uint8_t* const* ref_recon, const uint8_t* const* ref_meas,
                       const uint8_t* const* ref_mask, int32_t H, int32_t W, int64_t pitch,
                       const rfsr_me_params* me, const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8,
                       void* const* stage_events, void* workspace, size_t ws_bytes, void* stream,
                       const Part& part, int slot) {
    if (nref < 0 || nref > 3) return RFSR_EINVAL;
    if (nref > 0 && (!ref_recon || !ref_meas || !ref_mask)) return RFSR_EINVAL;
    if (stage_events)
        for (int k = 0; k < 4; ++k)
            if (!stage_events[k]) return RFSR_EINVAL;
    rfsr_frame_desc d;
    memset(&d, 0, sizeof(d));
    d.cur = cur;
    d.cur_mask = cur_mask;
    for (int k = 0; k < nref; ++k) {
        d.ref_recon[k] = ref_recon[k];
        d.ref_meas[k] = ref_meas[k];
        d.ref_mask[k] = ref_mask[k];
    }
    d.out = out;
    d.out_u8 = out_u8;
    d.nref = nref;
    d.H = H;
    d.W = W;
    d.pitch = pitch;
    rfsr_status st = check_frame(to_frame(d), part.finish());
    if (st != RFSR_OK) return st;
    if ((st = check_me(me)) != RFSR_OK) return st;
    if (part.finish() && (st = check_fsr(fsr)) != RFSR_OK) return st;
    const size_t scratch = single_ws(H, W, nref > 0 ? nref : 1);
    if ((st = check_ws(workspace, ws_bytes, scratch + kFrameTable * (size_t)(slot + 1))) != RFSR_OK) return st;
    if (!part.finish() && part.first >= nref) return RFSR_OK;   // nothing to run early

    uint8_t* ws = static_cast<uint8_t*>(workspace);
    const BatchLayout L(&d, 1);   // L.total <= scratch, L.table_bytes <= kFrameTable
    FrameTableImage img;
    write_image(&d, 1, *me, ws, L, reinterpret_cast<uint8_t*>(img.w), part);
    return from_hip(run_batch(&d, 1, *me, fsr, ws + scratch + kFrameTable * (size_t)slot, &img, stage_events,
                              ws, L, static_cast<hipStream_t>(stream), part));
}

// --------------------------------------------------------- static scratch --
// The scratch of fsr_blocks_noalloc: a file-scope device array, one copy per
// device (each GPU that runs the library holds its own until the process
// ends).  In host code `scratch` names a host-side stand-in, never the device
// memory: its device address is looked up once per device with that device
// current and kept in g_scratch; only that address is passed to kernels.
constexpr size_t kStaticScratch = RFSR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratch];
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device.
rfsr_status static_scratch(void** p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RFSR_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return RFSR_EDEVICE;
        g_scratch[dev] = q;
    }
    *p = g_scratch[dev];
    return RFSR_OK;
}

// Scratch bytes of one fsr_blocks call: the FSR tables, and for the mixed
// form the recomputation list.
size_t fsr_blocks_scratch_bytes(int H, int W, int precision) {
    return align256(sizeof(FsrTables)) +
           (precision == RFSR_PREC_MIXED ? rerun_bytes((size_t)(H / kBlock) * (W / kBlock)) : 0);
}

rfsr_status check_blocks_args(const float* values, const uint8_t* cls, int32_t H, int32_t W, int64_t pitch,
                              const rfsr_fsr_params* fsr, const float* out) {
    if (!values || !cls || !out) return RFSR_EINVAL;
    const rfsr_status st = check_shape(H, W, pitch);
    if (st != RFSR_OK) return st;
    return check_fsr(fsr);
}

// fsr_blocks on a validated request, its scratch (the FSR tables) at `workspace`.
rfsr_status run_fsr_blocks(const float* values, const uint8_t* cls, int32_t H, int32_t W, int64_t pitch,
                           const rfsr_fsr_params& fsr_p, float* out, uint8_t* out_u8, void* workspace,
                           size_t ws_bytes, void* stream) {
    const rfsr_fsr_params* fsr = &fsr_p;
    rfsr_status st = check_ws(workspace, ws_bytes, fsr_blocks_scratch_bytes(H, W, fsr->precision));
    if (st != RFSR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FsrTables* tab = static_cast<FsrTables*>(workspace);
    unsigned* rerun = fsr->precision == RFSR_PREC_MIXED
                          ? reinterpret_cast<unsigned*>(static_cast<uint8_t*>(workspace) + align256(sizeof(FsrTables)))
                          : nullptr;
    FrameJob fj;
    memset(&fj, 0, sizeof(fj));
    fj.values = const_cast<float*>(values);   // read only by the FSR kernel
    fj.cls = const_cast<uint8_t*>(cls);
    fj.out = out;
    fj.out_u8 = out_u8;
    fj.pitch = pitch;
    fj.opitch = pitch;
    fj.vpitch = pitch;
    fj.H = H;
    fj.W = W;
    hipError_t e = launch_fsr_tables(tab, fsr->rho, fsr->prior_sigma, s, rerun);
    if (e == hipSuccess) e = launch_fsr(single(fj), (H / kBlock) * (W / kBlock), *fsr, tab, s, nullptr, rerun);
    return from_hip(e);
}

}  // namespace

extern "C" {

size_t rfsr_workspace_bytes(int32_t H, int32_t W, int32_t nref, const rfsr_me_params* me,
                            const rfsr_fsr_params* fsr) {
    if (check_shape(H, W, W) != RFSR_OK || nref < 0 || nref > 3) return 0;
    if (me && check_me(me) == RFSR_EINVAL) return 0;
    if (fsr && check_fsr(fsr) == RFSR_EINVAL) return 0;
    return single_ws(H, W, nref > 0 ? nref : 1) + 2 * kFrameTable;
}

rfsr_status rfsr_motion_check(const uint8_t* cur, const uint8_t* cur_mask, const uint8_t* ref_recon,
                              int32_t H, int32_t W, int64_t pitch, const rfsr_me_params* me,
                              int8_t* mv, uint8_t* accept, uint16_t* cost,
                              unsigned long long* counters, void* workspace, size_t ws_bytes,
                              void* stream) {
    if (!cur || !cur_mask || !ref_recon || !mv || !accept) return RFSR_EINVAL;
    rfsr_status st = check_shape(H, W, pitch);
    if (st != RFSR_OK) return st;
    if ((st = check_me(me)) != RFSR_OK) return st;
    if ((st = check_ws(workspace, ws_bytes, single_ws(H, W, 1))) != RFSR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t* base = static_cast<uint8_t*>(workspace) + align256(sizeof(FsrTables));
    Frame f;
    memset(&f, 0, sizeof(f));
    f.cur = cur;
    f.cur_mask = cur_mask;
    f.ref_recon[0] = ref_recon;
    f.nref = 1;
    f.H = H;
    f.W = W;
    f.pitch = pitch;
    FrameJob fj;
    RefJob rj[3];
    const bool windows = check_needs_windows(me->check);
    make_jobs(f, base, windows, fj, rj);
    RefJob& j = rj[0];
    j.ref_mask = nullptr;   // decide every pixel
    j.mv_a = mv;            // outputs in the caller's planes (pitch)
    j.mv_b = mv + (int64_t)H * pitch;
    j.accept = accept;
    j.opitch = pitch;
    if (cost) {
        j.cost = cost;
        j.cpitch = pitch;
    }
    hipError_t e = launch_windows(single(fj), windows ? win_groups(H, W) : 0, s);
    if (e == hipSuccess)
        e = launch_motion(single(j), me_tiles(H, W), px_groups(H, W), frmc_groups(H, W), *me, counters, s);
    return from_hip(e);
}

rfsr_status fsr_blocks(const float* values, const uint8_t* cls, int32_t H, int32_t W, int64_t pitch,
                       const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8, void* workspace,
                       size_t ws_bytes, void* stream) {
    const rfsr_status st = check_blocks_args(values, cls, H, W, pitch, fsr, out);
    if (st != RFSR_OK) return st;
    return run_fsr_blocks(values, cls, H, W, pitch, *fsr, out, out_u8, workspace, ws_bytes, stream);
}

rfsr_status fsr_blocks_noalloc(const float* values, const uint8_t* cls, int32_t H, int32_t W, int64_t pitch,
                               const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8, void* stream) {
    rfsr_status st = check_blocks_args(values, cls, H, W, pitch, fsr, out);
    if (st != RFSR_OK) return st;
    if (fsr_blocks_scratch_bytes(H, W, fsr->precision) > kStaticScratch) return RFSR_EWORKSPACE;
    void* ws = nullptr;
    if ((st = static_scratch(&ws)) != RFSR_OK) return st;
    return run_fsr_blocks(values, cls, H, W, pitch, *fsr, out, out_u8, ws, kStaticScratch, stream);
}

rfsr_status rfsr_reconstruct_frame(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                                   const uint8_t* const* ref_recon, const uint8_t* const* ref_meas,
                                   const uint8_t* const* ref_mask, int32_t H, int32_t W,
                                   int64_t pitch, const rfsr_me_params* me,
                                   const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8,
                                   void* const* stage_events, void* workspace, size_t ws_bytes,
                                   void* stream) {
    return frame_call(cur, cur_mask, nref, ref_recon, ref_meas, ref_mask, H, W, pitch, me, fsr, out, out_u8,
                      stage_events, workspace, ws_bytes, stream, Part(), 0);
}

rfsr_status rfsr_frame_motion(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                              const uint8_t* const* ref_recon, const uint8_t* const* ref_meas,
                              const uint8_t* const* ref_mask, int32_t H, int32_t W, int64_t pitch,
                              const rfsr_me_params* me, int32_t first, void* workspace, size_t ws_bytes,
                              void* stream) {
    if (first < 0 || first > nref) return RFSR_EINVAL;
    return frame_call(cur, cur_mask, nref, ref_recon, ref_meas, ref_mask, H, W, pitch, me, nullptr, nullptr,
                      nullptr, nullptr, workspace, ws_bytes, stream, Part::motion(first), 1);
}

rfsr_status rfsr_frame_finish(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                              const uint8_t* const* ref_recon, const uint8_t* const* ref_meas,
                              const uint8_t* const* ref_mask, int32_t H, int32_t W, int64_t pitch,
                              const rfsr_me_params* me, const rfsr_fsr_params* fsr, int32_t first,
                              float* out, uint8_t* out_u8, void* const* stage_events, void* workspace,
                              size_t ws_bytes, void* stream) {
    if (first < 0 || first > nref) return RFSR_EINVAL;
    return frame_call(cur, cur_mask, nref, ref_recon, ref_meas, ref_mask, H, W, pitch, me, fsr, out, out_u8,
                      stage_events, workspace, ws_bytes, stream, Part::finish_from(first), 0);
}

size_t rfsr_batch_workspace_bytes(const rfsr_frame_desc* frames, int32_t n, const rfsr_me_params* me,
                                  const rfsr_fsr_params* fsr) {
    if (check_batch(frames, n) != RFSR_OK) return 0;
    if (me && check_me(me) == RFSR_EINVAL) return 0;
    if (fsr && check_fsr(fsr) == RFSR_EINVAL) return 0;
    return BatchLayout(frames, n).total;
}

size_t rfsr_batch_table_bytes(const rfsr_frame_desc* frames, int32_t n) {
    if (check_batch(frames, n) != RFSR_OK) return 0;
    return BatchLayout(frames, n).table_bytes;
}

rfsr_status rfsr_batch_write_tables_part(const rfsr_frame_desc* frames, int32_t n, const rfsr_me_params* me,
                                         int32_t part, int32_t first, const void* workspace, void* image,
                                         size_t image_bytes) {
    rfsr_status st = check_batch(frames, n);
    if (st != RFSR_OK) return st;
    if ((st = check_me(me)) != RFSR_OK) return st;
    if (part < RFSR_PART_ALL || part > RFSR_PART_FINISH || first < 0 || first > 3) return RFSR_EINVAL;
    if (!workspace || ((uintptr_t)workspace & 255u) != 0) return RFSR_EWORKSPACE;
    const BatchLayout L(frames, n);
    if (!image || image_bytes < L.table_bytes) return RFSR_EINVAL;
    Part pt;
    pt.kind = part;
    pt.first = part == RFSR_PART_ALL ? 0 : first;
    write_image(frames, n, *me, static_cast<uint8_t*>(const_cast<void*>(workspace)), L,
                static_cast<uint8_t*>(image), pt);
    return RFSR_OK;
}

rfsr_status rfsr_batch_write_tables(const rfsr_frame_desc* frames, int32_t n, const rfsr_me_params* me,
                                    const void* workspace, void* image, size_t image_bytes) {
    return rfsr_batch_write_tables_part(frames, n, me, RFSR_PART_ALL, 0, workspace, image, image_bytes);
}

rfsr_status rfsr_reconstruct_batch_part(const rfsr_frame_desc* frames, int32_t n, const rfsr_me_params* me,
                                        const rfsr_fsr_params* fsr, int32_t part, int32_t first,
                                        const void* job_tables, void* const* stage_events, void* workspace,
                                        size_t ws_bytes, void* stream) {
    rfsr_status st = check_batch(frames, n);
    if (st != RFSR_OK) return st;
    if ((st = check_me(me)) != RFSR_OK) return st;
    if (part < RFSR_PART_ALL || part > RFSR_PART_FINISH || first < 0 || first > 3) return RFSR_EINVAL;
    if (part != RFSR_PART_MOTION && (st = check_fsr(fsr)) != RFSR_OK) return st;
    if (!job_tables || ((uintptr_t)job_tables & 255u) != 0) return RFSR_EINVAL;
    if (stage_events)
        for (int k = 0; k < 4; ++k)
            if (!stage_events[k]) return RFSR_EINVAL;
    const BatchLayout L(frames, n);
    if ((st = check_ws(workspace, ws_bytes, L.total)) != RFSR_OK) return st;
    Part pt;
    pt.kind = part;
    pt.first = part == RFSR_PART_ALL ? 0 : first;
    return from_hip(run_batch(frames, n, *me, fsr, static_cast<const uint8_t*>(job_tables), nullptr,
                              stage_events, static_cast<uint8_t*>(workspace), L,
                              static_cast<hipStream_t>(stream), pt));
}

rfsr_status rfsr_reconstruct_batch(const rfsr_frame_desc* frames, int32_t n, const rfsr_me_params* me,
                                   const rfsr_fsr_params* fsr, const void* job_tables,
                                   void* const* stage_events, void* workspace, size_t ws_bytes,
                                   void* stream) {
    return rfsr_reconstruct_batch_part(frames, n, me, fsr, RFSR_PART_ALL, 0, job_tables, stage_events,
                                       workspace, ws_bytes, stream);
}

size_t rfsr_quality_workspace_bytes(int32_t H, int32_t W, int32_t border) {
    if (H <= 0 || W <= 0 || H > kMaxDim || W > kMaxDim || border < 0) return 0;
    if ((int64_t)H - 2 * (int64_t)border < 11 || (int64_t)W - 2 * (int64_t)border < 11) return 0;
    return align256(2 * sizeof(double) * (size_t)quality_tiles(H, W, border));
}

rfsr_status rfsr_quality(const uint8_t* ref, const float* test, int32_t H, int32_t W, int64_t pitch,
                         int32_t border, double* result, void* workspace, size_t ws_bytes, void* stream) {
    if (!ref || !test || !result) return RFSR_EINVAL;
    if (border < 0) return RFSR_EINVAL;
    if (H <= 0 || W <= 0 || H > kMaxDim || W > kMaxDim || pitch < W || pitch > (int64_t)1 << 30)
        return RFSR_ESHAPE;
    const size_t need = rfsr_quality_workspace_bytes(H, W, border);
    if (need == 0) return RFSR_ESHAPE;   // cropped frame smaller than one window
    rfsr_status st = check_ws(workspace, ws_bytes, need);
    if (st != RFSR_OK) return st;
    return from_hip(launch_quality(ref, test, H, W, pitch, border, static_cast<double*>(workspace), result,
                                   static_cast<hipStream_t>(stream)));
}

rfsr_status rfsr_event_create(void** event) {
    if (!event) return RFSR_EINVAL;
    hipEvent_t ev;
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) return RFSR_EDEVICE;
    *event = ev;
    return RFSR_OK;
}

rfsr_status rfsr_event_destroy(void* event) {
    if (!event) return RFSR_EINVAL;
    return from_hip(hipEventDestroy(static_cast<hipEvent_t>(event)));
}

rfsr_status rfsr_event_record(void* event, void* stream) {
    if (!event) return RFSR_EINVAL;
    return from_hip(hipEventRecord(static_cast<hipEvent_t>(event), static_cast<hipStream_t>(stream)));
}

rfsr_status rfsr_event_wait(void* event, void* stream) {
    if (!event) return RFSR_EINVAL;
    return from_hip(hipStreamWaitEvent(static_cast<hipStream_t>(stream), static_cast<hipEvent_t>(event), 0));
}

rfsr_status rfsr_event_elapsed_ms(void* start, void* stop, float* ms) {
    if (!start || !stop || !ms) return RFSR_EINVAL;
    hipError_t e = hipEventSynchronize(static_cast<hipEvent_t>(stop));
    if (e == hipSuccess) e = hipEventElapsedTime(ms, static_cast<hipEvent_t>(start), static_cast<hipEvent_t>(stop));
    return from_hip(e);
}

const char* rfsr_status_string(int32_t status) {
    switch (status) {
        case RFSR_OK: return "RFSR_OK";
        case RFSR_EINVAL: return "RFSR_EINVAL: invalid argument";
        case RFSR_ESHAPE: return "RFSR_ESHAPE: unsupported H, W or pitch";
        case RFSR_EWORKSPACE: return "RFSR_EWORKSPACE: workspace null, misaligned or too small";
        case RFSR_EDEVICE: return "RFSR_EDEVICE: HIP runtime error";
        case RFSR_EUNSUPPORTED: return "RFSR_EUNSUPPORTED: parameters not supported by this library";
        default: return "unknown rfsr status";
    }
}

int32_t rfsr_version(void) { return kVersion; }

}  // extern "C"

// C ABI of librfsr: argument validation, workspace layout, stage sequencing.
// Every step of the reconstruction runs in the kernels of fsr.hip and
// motion.hip; this file only validates, carves the caller's workspace and
// enqueues launches on the caller's stream.
#include <math.h>
#include <string.h>

#include "common.h"

using namespace rfsr;

namespace {

constexpr int32_t kVersion = 10000;   // 1.0.0

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
    if (p->block != kBlock || p->support != kSupport) return RFSR_EUNSUPPORTED;
    return RFSR_OK;
}

rfsr_status check_ws(void* ws, size_t have, size_t need) {
    if (!ws || ((uintptr_t)ws & 255u) != 0 || have < need) return RFSR_EWORKSPACE;
    return RFSR_OK;
}

// Frame workspace: FSR tables | motion scratch | per reference (mv_a, mv_b,
// accept) | FSR input values (f32) and classes (u8).  Planes use pitch W.
struct FrameLayout {
    size_t tables, motion, ref[3][3], values, cls, total;
    FrameLayout(int H, int W, int nref, const rfsr_me_params& me) {
        const size_t px = (size_t)H * W;
        size_t o = 0;
        tables = o; o = align256(o + sizeof(FsrTables));
        motion = o; o = align256(o + motion_ws_bytes(H, W, me));
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j) {
                ref[k][j] = o;
                if (k < nref) o = align256(o + px);
            }
        values = o; o = align256(o + 4 * px);
        cls = o; o = align256(o + px);
        total = o;
    }
};

}  // namespace

extern "C" {

size_t rfsr_workspace_bytes(int32_t H, int32_t W, int32_t nref, const rfsr_me_params* me,
                            const rfsr_fsr_params* fsr) {
    if (check_shape(H, W, W) != RFSR_OK || nref < 0 || nref > 3) return 0;
    rfsr_me_params mp = me ? *me : rfsr_me_params{4, 9, RFSR_CHECK_NNC_FRMC, 0};
    if (me && check_me(me) == RFSR_EINVAL) return 0;
    if (fsr && check_fsr(fsr) == RFSR_EINVAL) return 0;
    return FrameLayout(H, W, nref, mp).total;
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
    const size_t need = motion_ws_bytes(H, W, *me);
    if ((st = check_ws(workspace, ws_bytes, need)) != RFSR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int8_t* mv_b = mv + (int64_t)H * pitch;
    return from_hip(run_motion_check(cur, cur_mask, ref_recon, H, W, pitch, *me, mv, mv_b, pitch, accept,
                                     pitch, cost, pitch, counters, workspace, false, nullptr, s));
}

rfsr_status fsr_blocks(const float* values, const uint8_t* cls, int32_t H, int32_t W, int64_t pitch,
                       const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8, void* workspace,
                       size_t ws_bytes, void* stream) {
    if (!values || !cls || !out) return RFSR_EINVAL;
    rfsr_status st = check_shape(H, W, pitch);
    if (st != RFSR_OK) return st;
    if ((st = check_fsr(fsr)) != RFSR_OK) return st;
    if ((st = check_ws(workspace, ws_bytes, align256(sizeof(FsrTables)))) != RFSR_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    FsrTables* tab = static_cast<FsrTables*>(workspace);
    hipError_t e = launch_fsr_tables(tab, fsr->rho, s);
    if (e == hipSuccess) e = launch_fsr(values, cls, H, W, pitch, *fsr, tab, out, out_u8, pitch, s);
    return from_hip(e);
}

rfsr_status rfsr_reconstruct_frame(const uint8_t* cur, const uint8_t* cur_mask, int32_t nref,
                                   const uint8_t* const* ref_recon, const uint8_t* const* ref_meas,
                                   const uint8_t* const* ref_mask, int32_t H, int32_t W,
                                   int64_t pitch, const rfsr_me_params* me,
                                   const rfsr_fsr_params* fsr, float* out, uint8_t* out_u8,
                                   void* const* stage_events, void* workspace, size_t ws_bytes,
                                   void* stream) {
    if (!cur || !cur_mask || !out) return RFSR_EINVAL;
    if (nref < 0 || nref > 3) return RFSR_EINVAL;
    if (nref > 0) {
        if (!ref_recon || !ref_meas || !ref_mask) return RFSR_EINVAL;
        for (int k = 0; k < nref; ++k)
            if (!ref_recon[k] || !ref_meas[k] || !ref_mask[k]) return RFSR_EINVAL;
    }
    if (stage_events)
        for (int k = 0; k < 4; ++k)
            if (!stage_events[k]) return RFSR_EINVAL;
    rfsr_status st = check_shape(H, W, pitch);
    if (st != RFSR_OK) return st;
    if ((st = check_me(me)) != RFSR_OK) return st;
    if ((st = check_fsr(fsr)) != RFSR_OK) return st;
    const FrameLayout L(H, W, nref, *me);
    if ((st = check_ws(workspace, ws_bytes, L.total)) != RFSR_OK) return st;

    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t* base = static_cast<uint8_t*>(workspace);
    hipError_t e = hipSuccess;
    auto record = [&](int k) {
        if (stage_events && e == hipSuccess) e = hipEventRecord(static_cast<hipEvent_t>(stage_events[k]), s);
    };
    record(0);
    FsrTables* tab = reinterpret_cast<FsrTables*>(base + L.tables);
    if (e == hipSuccess) e = launch_fsr_tables(tab, fsr->rho, s);
    ProjRef refs[3];
    for (int k = 0; k < nref && e == hipSuccess; ++k) {
        int8_t* a = reinterpret_cast<int8_t*>(base + L.ref[k][0]);
        int8_t* b = reinterpret_cast<int8_t*>(base + L.ref[k][1]);
        uint8_t* acc = base + L.ref[k][2];
        e = run_motion_check(cur, cur_mask, ref_recon[k], H, W, pitch, *me, a, b, W, acc, W, nullptr, 0,
                             nullptr, base + L.motion, k > 0, ref_mask[k], s);
        refs[k] = ProjRef{a, b, acc, ref_meas[k], ref_mask[k]};
    }
    record(1);
    float* values = reinterpret_cast<float*>(base + L.values);
    uint8_t* cls = base + L.cls;
    if (e == hipSuccess) e = launch_project(cur, cur_mask, H, W, pitch, nref, refs, W, values, cls, s);
    record(2);
    // FSR reads values/cls (workspace, pitch W) and writes with the caller's pitch.
    if (e == hipSuccess) e = launch_fsr(values, cls, H, W, W, *fsr, tab, out, out_u8, pitch, s);
    record(3);
    return from_hip(e);
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
        case RFSR_EUNSUPPORTED: return "RFSR_EUNSUPPORTED: parameters not supported by this build";
        default: return "unknown rfsr status";
    }
}

int32_t rfsr_version(void) { return kVersion; }

}  // extern "C"

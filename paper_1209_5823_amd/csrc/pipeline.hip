// Streamed difference images of many host-resident tiles (Sec. 4: image data
// moves by asynchronous transfers between page-locked host memory and the
// device, on streams; Sec. 3: a mosaic camera delivers many equal tiles).
//
// A pipeline owns `depth` slots of device buffers (R, I/D, a) and three
// streams of default priority: copies in, compute, copies out.  Tile t uses
// slot t mod depth:
//   in:      wait out[slot] (its last tile is back on the host), copy R_t, I_t, a_t
//   compute: wait in[slot], D_t = R_t (x) K(a_t) - I_t written over I_t
//   out:     wait compute[slot], copy D_t to the host
// so the transfers of one tile overlap the contraction of the others.  The
// compute stream runs tiles in order, which also serialises the plan's
// per-call scratch (regrouped filters and their fragments).
#include <new>

#include "internal.hpp"

using namespace svc;

struct svconv_pipeline {
    svconv_plan* plan = nullptr;
    int depth = 0;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    std::vector<float*> dR, dID, dA;
    std::vector<hipEvent_t> ev_in, ev_comp, ev_out;
};

static void free_pipeline(svconv_pipeline* q) {
    for (auto v : {&q->dR, &q->dID, &q->dA})
        for (float* p : *v)
            if (p) (void)hipFree(p);
    for (auto v : {&q->ev_in, &q->ev_comp, &q->ev_out})
        for (hipEvent_t e : *v)
            if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : {q->s_in, q->s_comp, q->s_out})
        if (s) (void)hipStreamDestroy(s);
    delete q;
}

extern "C" {

int svconv_host_alloc(size_t bytes, void** out) {
    if (!out) return fail(SVCONV_EINVAL, "NULL argument");
    *out = nullptr;
    if (bytes == 0) return fail(SVCONV_EINVAL, "zero bytes");
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(SVCONV_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    *out = p;
    return SVCONV_OK;
}

int svconv_host_free(void* p) {
    if (!p) return SVCONV_OK;
    return hip_status(hipHostFree(p), "hipHostFree");
}

int svconv_pipeline_create(svconv_plan* plan, int depth, svconv_pipeline** out) {
    if (!out) return fail(SVCONV_EINVAL, "NULL argument");
    *out = nullptr;
    if (!plan) return fail(SVCONV_EINVAL, "plan is NULL");
    if (depth < 1 || depth > 8) return fail(SVCONV_EINVAL, "depth must be in [1, 8]");
    svconv_pipeline* q = new (std::nothrow) svconv_pipeline();
    if (!q) return fail(SVCONV_ENOMEM, "pipeline");
    q->plan = plan;
    q->depth = depth;
    q->dR.assign(depth, nullptr);
    q->dID.assign(depth, nullptr);
    q->dA.assign(depth, nullptr);
    q->ev_in.assign(depth, nullptr);
    q->ev_comp.assign(depth, nullptr);
    q->ev_out.assign(depth, nullptr);
    const size_t img = (size_t)plan->H * plan->W * sizeof(float);
    const size_t coef = (size_t)plan->N * plan->M * sizeof(float);
    int st = hip_status(hipStreamCreateWithFlags(&q->s_in, hipStreamNonBlocking), "stream");
    if (!st) st = hip_status(hipStreamCreateWithFlags(&q->s_comp, hipStreamNonBlocking), "stream");
    if (!st) st = hip_status(hipStreamCreateWithFlags(&q->s_out, hipStreamNonBlocking), "stream");
    for (int i = 0; i < depth && !st; ++i) {
        if (hipMalloc(&q->dR[i], img) != hipSuccess || hipMalloc(&q->dID[i], img) != hipSuccess ||
            hipMalloc(&q->dA[i], coef) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(SVCONV_ENOMEM, "pipeline slot buffers");
            break;
        }
        st = hip_status(hipEventCreateWithFlags(&q->ev_in[i], hipEventDisableTiming), "event");
        if (!st) st = hip_status(hipEventCreateWithFlags(&q->ev_comp[i], hipEventDisableTiming), "event");
        if (!st) st = hip_status(hipEventCreateWithFlags(&q->ev_out[i], hipEventDisableTiming), "event");
    }
    if (st) {
        free_pipeline(q);
        return st;
    }
    *out = q;
    return SVCONV_OK;
}

int svconv_pipeline_run(svconv_pipeline* q, int n_tiles, const float* const* R_host,
                        const float* const* I_host, const float* const* a_host,
                        float* const* D_host) {
    if (!q) return fail(SVCONV_EINVAL, "pipeline is NULL");
    if (n_tiles < 0) return fail(SVCONV_EINVAL, "n_tiles < 0");
    if (n_tiles == 0) return SVCONV_OK;
    if (!R_host || !I_host || !a_host || !D_host) return fail(SVCONV_EINVAL, "NULL argument");
    for (int t = 0; t < n_tiles; ++t)
        if (!R_host[t] || !I_host[t] || !a_host[t] || !D_host[t])
            return fail(SVCONV_EINVAL, "NULL tile pointer");
    svconv_plan* p = q->plan;
    const size_t img = (size_t)p->H * p->W * sizeof(float);
    const size_t coef = (size_t)p->N * p->M * sizeof(float);
    hipStream_t saved = p->stream;
    p->stream = q->s_comp;
    int st = SVCONV_OK;
    for (int t = 0; t < n_tiles && !st; ++t) {
        const int s = t % q->depth;
        if (t >= q->depth)
            st = hip_status(hipStreamWaitEvent(q->s_in, q->ev_out[s], 0), "wait");
        if (!st) st = hip_status(hipMemcpyAsync(q->dR[s], R_host[t], img, hipMemcpyHostToDevice, q->s_in), "copy R");
        if (!st) st = hip_status(hipMemcpyAsync(q->dID[s], I_host[t], img, hipMemcpyHostToDevice, q->s_in), "copy I");
        if (!st) st = hip_status(hipMemcpyAsync(q->dA[s], a_host[t], coef, hipMemcpyHostToDevice, q->s_in), "copy a");
        if (!st) st = hip_status(hipEventRecord(q->ev_in[s], q->s_in), "record");
        if (!st) st = hip_status(hipStreamWaitEvent(q->s_comp, q->ev_in[s], 0), "wait");
        if (!st) st = run_forward(p, q->dR[s], q->dID[s], q->dA[s], q->dID[s]);
        if (!st) st = hip_status(hipEventRecord(q->ev_comp[s], q->s_comp), "record");
        if (!st) st = hip_status(hipStreamWaitEvent(q->s_out, q->ev_comp[s], 0), "wait");
        if (!st) st = hip_status(hipMemcpyAsync(D_host[t], q->dID[s], img, hipMemcpyDeviceToHost, q->s_out), "copy D");
        if (!st) st = hip_status(hipEventRecord(q->ev_out[s], q->s_out), "record");
    }
    p->stream = saved;
    // drain every stream, also after an error, so no copy is left in flight
    int st2 = hip_status(hipStreamSynchronize(q->s_in), "synchronize");
    int st3 = hip_status(hipStreamSynchronize(q->s_comp), "synchronize");
    int st4 = hip_status(hipStreamSynchronize(q->s_out), "synchronize");
    if (st) return st;
    return st2 ? st2 : (st3 ? st3 : st4);
}

int svconv_pipeline_destroy(svconv_pipeline* q) {
    if (!q) return SVCONV_OK;
    int st = hip_status(hipStreamSynchronize(q->s_in), "synchronize");
    if (!st) st = hip_status(hipStreamSynchronize(q->s_comp), "synchronize");
    if (!st) st = hip_status(hipStreamSynchronize(q->s_out), "synchronize");
    free_pipeline(q);
    return st;
}

}  // extern "C"

// The serving session: scenes resident in device memory, requests admitted
// by the device memory their work needs, and their frames in flight on
// several streams at once (continuous batching).  Host code only; the frames
// run the same pyramid, trace and resolve kernels as ssr_shade.
//
// One worker thread per session owns the device side: it launches admitted
// requests on the stream of a free slot, records an event behind each, polls
// the events, and on completion returns the slot and the workspace and
// admits whatever waits.  Callers submit and poll from any thread; one mutex
// guards the session.
//
// A frame is the launch plan of ssr_shade (pyramid, counter reset, trace,
// resolve).  Each slot keeps one instantiated HIP graph per plan structure
// (the kernel, grid, block and shared memory of every launch: fixed by the
// image size, march mode and storage type), built from the plan as a chain
// of kernel nodes on the structure's first request; a later request of the
// same structure replaces the nodes' parameters in the instantiated graph
// and replays it.  A slot runs one request at a time, so its graphs are
// never updated while a launch of them is in flight.
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "kernels.h"
#include "scheduler.h"
#include "ssr.h"

namespace {

constexpr int64_t kAlign = 256;
int64_t round_up(int64_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

int64_t gbuf_elem(int dtype) { return dtype == SSR_F32 ? 16 : 8; }

// Workspace of one request: tile counter, depth pyramid (hierarchical
// march), per-sample hit codes.
struct Workspace {
    int64_t counter, hiz, codes, total;
};

Workspace workspace_of(const ssr_camera& cam, const ssr_params& p, const ssr::HizLayout& lay) {
    Workspace w;
    w.counter = 0;
    w.hiz = kAlign;
    const int64_t hiz_bytes = p.march == SSR_MARCH_HIZ ? round_up(lay.total * 16) : 0;
    w.codes = w.hiz + hiz_bytes;
    w.total = w.codes + ssr_codes_count(cam.width, cam.height, p.spp, p.flags | SSR_CODES_TILED) * 4;
    return w;
}

}  // namespace

struct ssr_session {
    struct Scene {
        ssr_camera cam;
        int32_t dtype;
        void* block;            // one allocation holding everything below
        float* depth;
        void *normal_rough, *albedo_metal, *radiance;
        float* env;
        int32_t env_w, env_h;
        float4* mips;
        int64_t bytes;
    };
    struct Record {
        ssr_request req;
        int64_t bytes;
        double t_submit = 0, t_admit = 0, t_done = 0;
        int status = SSR_PENDING;
    };
    // A plan's structure: per launch, kernel, grid, block, shared memory.
    using Shape = std::vector<uint64_t>;
    struct Graph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        std::vector<hipGraphNode_t> nodes;   // one kernel node per launch, in plan order
    };
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        std::map<Shape, Graph> graphs;
    };

    int device = 0;
    int cu_count = 1;
    ssr_session_cfg cfg;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work;   // the worker: something to admit, or stop
    std::condition_variable cv_done;   // waiters: a request finished
    std::thread worker;
    bool stop = false;
    bool serving = false;              // the first submit has set up the arena and slots

    std::vector<Scene> scenes;
    int64_t scene_bytes = 0;
    char* arena = nullptr;
    std::unique_ptr<ssr::serve::Scheduler> sched;
    std::vector<Slot> slots;
    std::unordered_map<uint64_t, Record> recs;
    uint64_t next_ticket = 1;
    int64_t completed = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void run();
    int launch(const ssr::serve::Admitted& ad);
    int replay(Slot& slot, ssr::Plan& plan);
};

namespace {

ssr_session::Shape shape_of(const ssr::Plan& plan) {
    ssr_session::Shape k;
    for (int i = 0; i < plan.n; ++i) {
        const ssr::Launch& x = plan.l[i];
        k.push_back(reinterpret_cast<uint64_t>(x.func));
        k.push_back((static_cast<uint64_t>(x.grid.x) << 32) | x.grid.y);
        k.push_back((static_cast<uint64_t>(x.block.x) << 32) | x.shmem);
    }
    return k;
}

hipKernelNodeParams node_params(ssr::Launch& x, void** argv) {
    x.argv(argv);
    hipKernelNodeParams p = {};
    p.func = const_cast<void*>(x.func);
    p.gridDim = x.grid;
    p.blockDim = x.block;
    p.sharedMemBytes = x.shmem;
    p.kernelParams = argv;
    p.extra = nullptr;
    return p;
}

}  // namespace

// Run `plan` on the slot's stream through its graph for the plan's structure
// (built and instantiated on first use, else updated node by node).
int ssr_session::replay(Slot& slot, ssr::Plan& plan) {
    const Shape key = shape_of(plan);
    auto it = slot.graphs.find(key);
    if (it == slot.graphs.end()) {
        Graph g;
        if (hipGraphCreate(&g.graph, 0) != hipSuccess) return SSR_E_HIP;
        hipGraphNode_t prev = nullptr;
        for (int i = 0; i < plan.n; ++i) {
            void* argv[ssr::kLaunchMaxArgs];
            const hipKernelNodeParams p = node_params(plan.l[i], argv);
            hipGraphNode_t node = nullptr;
            if (hipGraphAddKernelNode(&node, g.graph, prev ? &prev : nullptr, prev ? 1 : 0, &p) !=
                hipSuccess) {
                (void)hipGraphDestroy(g.graph);
                return SSR_E_HIP;
            }
            g.nodes.push_back(node);
            prev = node;
        }
        if (hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return SSR_E_HIP;
        }
        it = slot.graphs.emplace(key, g).first;
    } else {
        for (int i = 0; i < plan.n; ++i) {
            void* argv[ssr::kLaunchMaxArgs];
            const hipKernelNodeParams p = node_params(plan.l[i], argv);
            if (hipGraphExecKernelNodeSetParams(it->second.exec, it->second.nodes[i], &p) !=
                hipSuccess)
                return SSR_E_HIP;
        }
    }
    return hipGraphLaunch(it->second.exec, slot.stream) == hipSuccess ? SSR_OK : SSR_E_HIP;
}

// Launch one admitted request on its slot's stream (mutex held).
int ssr_session::launch(const ssr::serve::Admitted& ad) {
    Record& rec = recs[ad.ticket];
    const Scene& sc = scenes[rec.req.scene_id];
    const ssr_params& p = rec.req.params;
    ssr_gbuffer g{sc.depth, sc.normal_rough, sc.albedo_metal, sc.radiance, sc.dtype, nullptr};
    ssr_env e{sc.env, sc.env_w, sc.env_h, reinterpret_cast<const float*>(sc.mips)};
    ssr::ShadeArgs a;
    ssr::EnvLayout el;
    ssr::HizLayout hl;
    if (ssr::fill_args(&sc.cam, &g, &e, &p, true, &a, &el, &hl) != SSR_OK) return SSR_E_ARG;
    const Workspace w = workspace_of(sc.cam, p, hl);
    char* ws = arena + ad.offset;
    const hipStream_t s = slots[ad.slot].stream;
    a.env = sc.mips;
    a.tile_counter = reinterpret_cast<int*>(ws + w.counter);
    a.codes = reinterpret_cast<int32_t*>(ws + w.codes);
    a.flags |= SSR_CODES_TILED;  // the request's own codes: tile-major, as ssr_shade's
    a.out = rec.req.out_rgb;
    // the frame's launches: those of ssr_shade with the request's workspace
    // (the plan lives on the heap: it holds a copy of every launch's arguments)
    std::unique_ptr<ssr::Plan> plan(new (std::nothrow) ssr::Plan);
    if (!plan) return SSR_E_NOMEM;
    if (p.march == SSR_MARCH_HIZ) {
        float4* hiz = reinterpret_cast<float4*>(ws + w.hiz);
        ssr::plan_hiz(sc.depth, hl, p.thickness, hiz, *plan);
        a.hiz = hiz;
    }
    ssr::plan_trace(a, sc.dtype, p.march, cu_count, *plan, /*overlapped=*/true);
    ssr::plan_resolve(a, sc.dtype, *plan);
    if (cfg.flags & SSR_SESSION_DIRECT) {
        if (ssr::run_plan(*plan, s) != hipSuccess) return SSR_E_HIP;
    } else {
        const int st = replay(slots[ad.slot], *plan);
        if (st != SSR_OK) return st;
    }
    if (hipEventRecord(slots[ad.slot].done, s) != hipSuccess) return SSR_E_HIP;
    return SSR_OK;
}

void ssr_session::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (stop) return;
        bool finished = false;
        for (int s = 0; s < sched->slots(); ++s) {
            if (!sched->busy(s)) continue;
            const hipError_t q = hipEventQuery(slots[s].done);
            if (q == hipErrorNotReady) continue;
            Record& rec = recs[sched->ticket_in(s)];
            rec.t_done = now();
            rec.status = q == hipSuccess ? SSR_OK : SSR_E_HIP;
            if (q != hipSuccess) (void)hipGetLastError();
            sched->finish(s);
            ++completed;
            finished = true;
        }
        for (const auto& ad : sched->admit()) {
            Record& rec = recs[ad.ticket];
            rec.t_admit = now();
            const int st = launch(ad);
            if (st != SSR_OK) {
                // nothing (more) was enqueued behind a failed launch: the slot
                // is released once the stream has drained what was
                (void)hipGetLastError();
                (void)hipStreamSynchronize(slots[ad.slot].stream);
                rec.t_done = now();
                rec.status = st;
                sched->finish(ad.slot);
                ++completed;
                finished = true;
            }
        }
        if (finished) cv_done.notify_all();
        if (sched->idle()) {
            cv_work.wait(lk, [this] { return stop || !sched->idle(); });
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

extern "C" {

int ssr_session_create(int device, const ssr_session_cfg* cfg, ssr_session** out) {
    if (!out) return SSR_E_ARG;
    *out = nullptr;
    if (!cfg || cfg->hbm_budget_bytes <= 0 || cfg->max_slots < 1 || cfg->max_slots > 64 ||
        cfg->max_bypass < 0 || (cfg->flags & ~static_cast<uint32_t>(SSR_SESSION_DIRECT)))
        return SSR_E_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return SSR_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return SSR_E_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SSR_E_DEVICE;
    ssr_session* s = new (std::nothrow) ssr_session;
    if (!s) return SSR_E_NOMEM;
    s->device = device;
    s->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return SSR_OK;
}

int ssr_session_add_scene(ssr_session* s, const ssr_camera* cam, const ssr_gbuffer* g,
                          const ssr_env* env, int32_t* scene_id, void* stream) {
    if (!s || !scene_id) return SSR_E_ARG;
    ssr_params probe{1, SSR_MARCH_HIZ, 1, 1.0f, 1.0f, 0.0f, 0, 0, 0};
    ssr::ShadeArgs a;
    ssr::EnvLayout el;
    ssr::HizLayout hl;
    int st = ssr::fill_args(cam, g, env, &probe, true, &a, &el, &hl);
    if (st == 1) return SSR_E_ARG;   // an empty image is not a scene
    if (st != SSR_OK) return st;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->serving) return SSR_E_BUSY;
    const int64_t px = static_cast<int64_t>(cam->width) * cam->height;
    const int64_t o_depth = 0, o_nr = round_up(px * 4), o_am = o_nr + round_up(px * gbuf_elem(g->dtype));
    const int64_t o_rad = o_am + round_up(px * gbuf_elem(g->dtype));
    const int64_t o_env = o_rad + round_up(px * gbuf_elem(g->dtype));
    const int64_t env_bytes = static_cast<int64_t>(env->width) * env->height * 12;
    const int64_t o_mips = o_env + round_up(env_bytes);
    const int64_t bytes = o_mips + round_up(el.total * 16);
    if (s->scene_bytes + bytes > s->cfg.hbm_budget_bytes) return SSR_E_BUDGET;
    if (hipSetDevice(s->device) != hipSuccess) return SSR_E_HIP;
    void* block = nullptr;
    if (hipMalloc(&block, static_cast<size_t>(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return SSR_E_NOMEM;
    }
    char* b = static_cast<char*>(block);
    const hipStream_t hs = static_cast<hipStream_t>(stream);
    const size_t gb = static_cast<size_t>(px * gbuf_elem(g->dtype));
    bool ok = hipMemcpyAsync(b + o_depth, g->depth, static_cast<size_t>(px * 4), hipMemcpyDeviceToDevice, hs) == hipSuccess &&
              hipMemcpyAsync(b + o_nr, g->normal_rough, gb, hipMemcpyDeviceToDevice, hs) == hipSuccess &&
              hipMemcpyAsync(b + o_am, g->albedo_metal, gb, hipMemcpyDeviceToDevice, hs) == hipSuccess &&
              hipMemcpyAsync(b + o_rad, g->radiance, gb, hipMemcpyDeviceToDevice, hs) == hipSuccess &&
              hipMemcpyAsync(b + o_env, env->rgb, static_cast<size_t>(env_bytes), hipMemcpyDeviceToDevice, hs) == hipSuccess;
    // the mip chain from the session's copy of the map
    ok = ok && ssr::launch_env_mips(reinterpret_cast<float*>(b + o_env), el,
                                    reinterpret_cast<float4*>(b + o_mips), hs) == hipSuccess;
    ok = ok && hipStreamSynchronize(hs) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        (void)hipFree(block);
        return SSR_E_HIP;
    }
    ssr_session::Scene sc;
    sc.cam = *cam;
    sc.dtype = g->dtype;
    sc.block = block;
    sc.depth = reinterpret_cast<float*>(b + o_depth);
    sc.normal_rough = b + o_nr;
    sc.albedo_metal = b + o_am;
    sc.radiance = b + o_rad;
    sc.env = reinterpret_cast<float*>(b + o_env);
    sc.env_w = env->width;
    sc.env_h = env->height;
    sc.mips = reinterpret_cast<float4*>(b + o_mips);
    sc.bytes = bytes;
    s->scenes.push_back(sc);
    s->scene_bytes += bytes;
    *scene_id = static_cast<int32_t>(s->scenes.size() - 1);
    return SSR_OK;
}

int64_t ssr_session_request_bytes(ssr_session* s, const ssr_request* r) {
    if (!s || !r) return -1;
    std::lock_guard<std::mutex> lk(s->mu);
    if (r->scene_id < 0 || r->scene_id >= static_cast<int32_t>(s->scenes.size())) return -1;
    ssr::HizLayout hl;
    const ssr_camera& cam = s->scenes[r->scene_id].cam;
    if (!ssr::make_hiz_layout(cam.width, cam.height, &hl)) return -1;
    return round_up(workspace_of(cam, r->params, hl).total);
}

int ssr_session_submit(ssr_session* s, const ssr_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket || !r->out_rgb) return SSR_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop) return SSR_E_BUSY;
    if (r->scene_id < 0 || r->scene_id >= static_cast<int32_t>(s->scenes.size())) return SSR_E_ARG;
    const ssr_session::Scene& sc = s->scenes[r->scene_id];
    ssr_gbuffer g{sc.depth, sc.normal_rough, sc.albedo_metal, sc.radiance, sc.dtype, nullptr};
    ssr_env e{sc.env, sc.env_w, sc.env_h, reinterpret_cast<const float*>(sc.mips)};
    ssr::ShadeArgs a;
    ssr::EnvLayout el;
    ssr::HizLayout hl;
    const int st = ssr::fill_args(&sc.cam, &g, &e, &r->params, true, &a, &el, &hl);
    if (st != SSR_OK) return st == 1 ? SSR_E_ARG : st;
    const int64_t bytes = workspace_of(sc.cam, r->params, hl).total;
    if (!s->serving) {
        // the first request: the rest of the budget becomes the workspace arena
        const int64_t cap = (s->cfg.hbm_budget_bytes - s->scene_bytes) / kAlign * kAlign;
        if (cap <= 0) return SSR_E_BUDGET;
        if (hipSetDevice(s->device) != hipSuccess) return SSR_E_HIP;
        if (hipMalloc(reinterpret_cast<void**>(&s->arena), static_cast<size_t>(cap)) != hipSuccess) {
            (void)hipGetLastError();
            s->arena = nullptr;
            return SSR_E_NOMEM;
        }
        s->slots.resize(s->cfg.max_slots);
        for (auto& sl : s->slots) {
            if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return SSR_E_HIP;
            }
        }
        s->sched.reset(new ssr::serve::Scheduler(cap, s->cfg.max_slots, s->cfg.max_bypass));
        s->serving = true;
        s->worker = std::thread([s] { s->run(); });
    }
    if (!s->sched->fits_ever(bytes)) return SSR_E_BUDGET;
    const uint64_t t = s->next_ticket++;
    ssr_session::Record rec;
    rec.req = *r;
    rec.bytes = s->sched->workspace(bytes);
    rec.t_submit = s->now();
    s->recs[t] = rec;
    s->sched->push(t, bytes);
    *ticket = t;
    lk.unlock();
    s->cv_work.notify_one();
    return SSR_OK;
}

static int fill_result(ssr_session* s, uint64_t ticket, ssr_result* res, bool wait) {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->recs.find(ticket);
    if (it == s->recs.end()) return SSR_E_TICKET;
    if (wait)
        s->cv_done.wait(lk, [&] { return s->stop || s->recs[ticket].status != SSR_PENDING; });
    const ssr_session::Record& rec = s->recs[ticket];
    if (rec.status == SSR_PENDING) return SSR_PENDING;
    if (res) {
        res->status = rec.status;
        res->t_submit = rec.t_submit;
        res->t_admit = rec.t_admit;
        res->t_done = rec.t_done;
        res->workspace_bytes = rec.bytes;
    }
    s->recs.erase(ticket);
    return SSR_OK;
}

int ssr_session_poll(ssr_session* s, uint64_t ticket, ssr_result* res) {
    if (!s) return SSR_E_ARG;
    return fill_result(s, ticket, res, false);
}

int ssr_session_wait(ssr_session* s, uint64_t ticket, ssr_result* res) {
    if (!s) return SSR_E_ARG;
    return fill_result(s, ticket, res, true);
}

int ssr_session_get_stats(ssr_session* s, ssr_session_stats* out) {
    if (!s || !out) return SSR_E_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    out->scene_bytes = s->scene_bytes;
    out->arena_bytes = s->sched ? s->sched->arena().capacity() : 0;
    out->arena_used = s->sched ? s->sched->arena().used() : 0;
    out->running = s->sched ? s->sched->running() : 0;
    out->waiting = s->sched ? s->sched->waiting() : 0;
    out->completed = s->completed;
    return SSR_OK;
}

void ssr_session_destroy(ssr_session* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        if (s->sched) s->sched->drop_waiting();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (hipSetDevice(s->device) == hipSuccess) {
        for (auto& sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            for (auto& kv : sl.graphs) {
                if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
                if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
            }
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        if (s->arena) (void)hipFree(s->arena);
        for (auto& sc : s->scenes) (void)hipFree(sc.block);
    }
    delete s;
}

}  // extern "C"

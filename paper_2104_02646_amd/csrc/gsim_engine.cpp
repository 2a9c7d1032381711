// Serving engine: continuous batching of system-identification gradient queries.
//
// A query is one body (tet mesh or cloth) with parameters, a start state, a
// target and a step count; its answer is the loss of the rollout's final
// positions and the gradients of that loss (App. A adjoint through the App. A.2
// semi-implicit Euler steps).  The engine
//   - admits queued queries in FIFO order while their exact device footprint
//     fits in the caller-owned pool (first-fit allocator over the pool);
//   - keeps every admitted query's states, checkpoints, segment buffer,
//     adjoint states, parameters and gradients on the device;
//   - advances every live query by one micro-step per tick, and runs the
//     micro-steps of all live queries together: one element pass and one
//     particle pass over the union of their tiles for the forward micro-steps,
//     and the same for the adjoint micro-steps.  A query's arithmetic and
//     reduction order do not depend on who else is in the batch.
// Per-query micro-steps: T forward steps (checkpoint every K), the loss seed,
// then for each checkpoint segment in reverse the recomputed forward steps and
// the adjoint steps, then the contact-gradient reduction and the copy-out.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstring>
#include <deque>
#include <memory>
#include <new>

#include "gsim_host.h"

using namespace gsim;

namespace {

#define HIP_TRY(call, what)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(e_, what);     \
    } while (0)

#define LAUNCH_TRY(call, what)                               \
    do {                                                     \
        int rc_ = (call);                                    \
        if (rc_) return hip_fail((hipError_t)rc_, what);     \
    } while (0)

size_t aup(size_t v) { return (v + 255) / 256 * 256; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device buffers of one query, as offsets from its pool region.
struct QLayout {
    size_t ws, ws_bytes, ckpt, seg, s0, sA, sB, seed, aA, aB, target, tiles;
    size_t mu, lam, ktri, mass, contact, g_mu, g_lam, g_ktri, g_mass, g_contact, loss;
    size_t total;
};

QLayout qlayout(const gsim_plan* P, int T, int K) {
    QLayout L;
    size_t ws = 0, ck = 0, sg = 0;
    gsim_plan_sizes(P, T, K, &ws, &ck, &sg);
    const size_t st = 6 * (size_t)P->np * 4;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t at = o;
        o = aup(o + b);
        return at;
    };
    L.ws_bytes = ws;
    L.ws = take(ws);
    L.ckpt = take(ck);
    L.seg = take(sg);
    L.s0 = take(st);
    L.sA = take(st);
    L.sB = take(st);
    L.seed = take(st);
    L.aA = take(st);
    L.aB = take(st);
    L.target = take(3 * (size_t)P->np * 4);
    // the query's element and particle tiles, resident while it is live (the particle
    // tiles of the default 256-particle tile size: one per started 256 of its particles)
    L.tiles = take(sizeof(Tile) * (P->etiles.size() + (size_t)((P->np + 255) / 256) + 1));
    L.mu = take(P->ne * 4);
    L.lam = take(P->ne * 4);
    L.ktri = take(P->nt * 4);
    L.mass = take(P->np * 4);
    L.contact = take(16);
    L.g_mu = take(P->ne * 4);
    L.g_lam = take(P->ne * 4);
    L.g_ktri = take(P->nt * 4);
    L.g_mass = take(P->np * 4);
    L.g_contact = take(16);
    L.loss = take(4);
    L.total = o;
    return L;
}

enum Phase { PH_FWD = 0, PH_LOSS = 1, PH_BWD = 2, PH_FIN = 3 };
enum OpKind { OP_NONE = 0, OP_FWD = 1, OP_ADJ = 2, OP_LOSS = 3, OP_FIN = 4 };

struct Query {
    int64_t id = 0;
    std::unique_ptr<gsim_plan, int (*)(gsim_plan*)> plan{nullptr, gsim_plan_destroy};
    int T = 0, K = 1;
    int64_t np = 0, ne = 0, nt = 0;
    std::vector<float> mu, lam, ktri, mass, contact, x0v0, target;  // x0v0 = [x0 | v0] SoA
    std::vector<Tile> tiles;  // element then particle tiles (kept for the upload's source)
    int n_etiles = 0, n_ptiles = 0;
    float *o_mu = nullptr, *o_lam = nullptr, *o_ktri = nullptr, *o_mass = nullptr, *o_contact = nullptr;
    QLayout lay{};
    double t_submit = 0;
};

struct Live {
    std::unique_ptr<Query> q;
    gsim_model* model = nullptr;
    size_t off = 0;  // pool region
    char* base = nullptr;
    int phase = PH_FWD;
    int t = 0;         // forward step
    int seg = 0;       // current backward segment
    int j = 0;         // recompute index inside the segment (j < L-1), then adjoint
    int ta = 0;        // next adjoint step
    int qa = 0;        // adjoint steps done
    double t_admit = 0;
    float* F(size_t o) const { return reinterpret_cast<float*>(base + o); }
};

struct Done {
    int64_t id;
    float loss;
    double t_submit, t_admit, t_done;
    int status;
};

// First-fit allocator over [0, size) with 256-byte granularity.
struct Pool {
    size_t size = 0;
    std::vector<std::pair<size_t, size_t>> free_list;  // (offset, length), sorted by offset
    void init(size_t s) {
        size = s;
        free_list.assign(1, {0, s});
    }
    bool alloc(size_t n, size_t& off) {
        n = aup(n);
        for (size_t i = 0; i < free_list.size(); ++i)
            if (free_list[i].second >= n) {
                off = free_list[i].first;
                free_list[i].first += n;
                free_list[i].second -= n;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = aup(n);
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        it = free_list.insert(it, {off, n});
        // merge with neighbours
        size_t i = it - free_list.begin();
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + i);
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto& f : free_list) s += f.second;
        return s;
    }
};

const int RING = 4;  // tick tables in flight
const size_t STAGE_CHUNK_BYTES = 8 << 20;  // per staging chunk (host and device), 4 chunks
const size_t RESULT_RING_BYTES = 32 << 20;  // pinned ring of results on their way out

// Staging of the queries' set-up copies: a ring of chunks, each a pinned host buffer
// and its device mirror.  copy() packs the bytes into the current chunk (16-byte
// aligned) and records the pieces; flush() appends the piece table, moves the chunk to
// its mirror with one copy and scatters it with one k_stage_copy launch, then moves to
// the next chunk once the launch that last read it has completed.  A copy larger than
// a chunk goes directly (and waits for the stream, since its source is the caller's).
struct Stager final : UploadSink {
    static const int N = 4;
    size_t cap = 0;
    char* host[N] = {};
    char* dev[N] = {};
    hipEvent_t evt[N] = {};
    hipStream_t stream = nullptr;
    int cur = 0;
    size_t fill = 0;
    std::vector<StageSeg> segs;
    int64_t flushes = 0, direct = 0;

    static size_t pieces(size_t n) { return (n + STAGE_PIECE - 1) / STAGE_PIECE; }
    size_t table_end(size_t data, size_t more) const {
        return (data + 15) / 16 * 16 + (segs.size() + more) * sizeof(StageSeg);
    }
    void add(const char* src, char* dst, size_t n) {
        for (size_t o = 0; o < n; o += (size_t)STAGE_PIECE)
            segs.push_back({src ? src + o : nullptr, dst + o, (int64_t)std::min((size_t)STAGE_PIECE, n - o)});
    }
    hipError_t copy(void* dst, const void* src, size_t n) override {
        if (n == 0) return hipSuccess;
        const size_t need = (n + 15) / 16 * 16;
        if (need + (pieces(n) + 1) * sizeof(StageSeg) > cap) {
            ++direct;
            hipError_t e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, stream);
            return e == hipSuccess ? hipStreamSynchronize(stream) : e;
        }
        if (table_end(fill + need, pieces(n)) > cap)
            if (hipError_t e = flush()) return e;
        std::memcpy(host[cur] + fill, src, n);
        add(dev[cur] + fill, (char*)dst, n);
        fill += need;
        return hipSuccess;
    }
    hipError_t zero(void* dst, size_t n) override {
        if (n == 0) return hipSuccess;
        if ((pieces(n) + 1) * sizeof(StageSeg) > cap) {
            ++direct;
            return hipMemsetAsync(dst, 0, n, stream);  // (the engine's stream is never captured)
        }
        if (table_end(fill, pieces(n)) > cap)
            if (hipError_t e = flush()) return e;
        add(nullptr, (char*)dst, n);
        return hipSuccess;
    }
    hipError_t flush() {
        if (segs.empty()) return hipSuccess;
        const size_t t0 = (fill + 15) / 16 * 16;
        std::memcpy(host[cur] + t0, segs.data(), segs.size() * sizeof(StageSeg));
        hipError_t e = hipMemcpyAsync(dev[cur], host[cur], table_end(fill, 0), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = (hipError_t)launch_stage_copy(reinterpret_cast<const StageSeg*>(dev[cur] + t0), (int)segs.size(), stream);
        if (e == hipSuccess) e = hipEventRecord(evt[cur], stream);
        cur = (cur + 1) % N;
        fill = 0;
        segs.clear();
        ++flushes;
        if (e == hipSuccess) e = hipEventSynchronize(evt[cur]);  // the chunk's last reader has finished
        return e;
    }
};

// A finished query whose results are on their way to a pinned ring: its gradient
// block [g_mu, loss] and status words land at [off, off + bytes) of the ring; `evt`
// (recorded after the copies of the round that finished it) says when.
struct Pending {
    std::unique_ptr<Query> q;
    size_t off = 0, bytes = 0, flags_at = 0;
    double t_admit = 0;
    hipEvent_t evt = nullptr;
};

// The pinned result ring: allocations in FIFO order, freed from the front.
struct ResultRing {
    char* host = nullptr;
    size_t cap = 0;
    size_t head = 0;
    std::deque<Pending> q;
    std::vector<hipEvent_t> free_events;

    bool place(size_t n, size_t& off) {
        if (n > cap) return false;
        if (q.empty()) {
            off = 0;
            head = n;
            return true;
        }
        const size_t tail = q.front().off;
        if (head > tail) {  // live entries [tail, head): free space after head and before tail
            if (head + n <= cap) {
                off = head;
                head += n;
                return true;
            }
            if (n < tail) {
                off = 0;
                head = n;
                return true;
            }
            return false;
        }
        if (head + n < tail) {  // wrapped: live [tail, cap) and [0, head), free [head, tail)
            off = head;
            head += n;
            return true;
        }
        return false;
    }
};

}  // namespace

struct gsim_engine {
    char* pool_base = nullptr;
    Pool pool;
    int max_live = 0;
    int64_t max_tiles = 0;
    hipStream_t stream = nullptr;
    // per-tick table ring: device blobs (carved from the pool) and pinned host copies
    size_t blob_bytes = 0, head_bytes = 0;
    char* blob_dev[RING] = {};
    char* blob_host[RING] = {};
    hipEvent_t blob_evt[RING] = {};
    int ring = 0;
    int64_t next_id = 1;
    std::deque<std::unique_ptr<Query>> queue;
    std::vector<Live> live;
    std::vector<Done> done;
    int micro_per_tick = 1;  // micro-step rounds per gsim_engine_tick
    size_t store_limit = 0;  // queries whose every-state footprint fits store every state
    int64_t ticks = 0, admitted = 0, completed = 0;  // ticks: micro-step rounds
    double live_sum = 0;  // sum over ticks of live queries (mean concurrency)
    Stager stage;         // the queries' set-up copies
    ResultRing results;   // finished queries' results on their way to the host
    bool round_finished = false;  // the current round issued result copies
};

namespace {

// Builds and uploads the device buffers of an admitted query.
int admit(gsim_engine* E, std::unique_ptr<Query>& q, size_t off) {
    Live L;
    L.off = off;
    L.base = E->pool_base + off;
    const QLayout& ly = q->lay;
    Stager& st = E->stage;
    int rc = model_init<float>(q->plan.get(), q->T, q->K, L.base + ly.ws, ly.ws_bytes, E->stream, &L.model, &st);
    if (rc) return rc;
    auto up = [&](size_t o, const std::vector<float>& v) -> hipError_t {
        if (v.empty()) return hipSuccess;
        return st.copy(L.base + o, v.data(), v.size() * 4);
    };
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    chk(up(ly.s0, q->x0v0));
    chk(up(ly.target, q->target));
    chk(up(ly.mu, q->mu));
    chk(up(ly.lam, q->lam));
    chk(up(ly.ktri, q->ktri));
    chk(up(ly.mass, q->mass));
    chk(up(ly.contact, q->contact));
    {
        const gsim_model* m = L.model;
        const size_t ne = m->etiles_nat.size(), npt = m->ptiles_nat.size();
        if (sizeof(Tile) * (ne + npt) > sizeof(Tile) * (q->plan->etiles.size() + (size_t)((q->np + 255) / 256) + 1))
            e = hipErrorInvalidValue;  // (cannot happen: the model keeps the default particle tile size)
        else if (ne + npt) {
            q->tiles.assign(m->etiles_nat.begin(), m->etiles_nat.end());
            q->tiles.insert(q->tiles.end(), m->ptiles_nat.begin(), m->ptiles_nat.end());
            chk(st.copy(L.base + ly.tiles, q->tiles.data(), sizeof(Tile) * q->tiles.size()));
            q->n_etiles = (int)ne;
            q->n_ptiles = (int)npt;
        }
    }
    if (e != hipSuccess) {
        gsim_model_destroy(L.model);
        return hip_fail(e, "upload query");
    }
    // zero gradients and contact partial rows
    const ModelDev<float>* md = reinterpret_cast<const ModelDev<float>*>(L.model->md_host.data());
    chk(st.zero(L.F(ly.g_mu), 4 * (size_t)q->ne));
    chk(st.zero(L.F(ly.g_lam), 4 * (size_t)q->ne));
    chk(st.zero(L.F(ly.g_ktri), 4 * (size_t)q->nt));
    chk(st.zero(L.F(ly.g_mass), 4 * (size_t)q->np));
    chk(st.zero(L.F(ly.g_contact), 16));
    chk(st.zero(md->cpart, 16 * (size_t)(L.model->n_ptile_rows + 1)));
    if (e != hipSuccess) {
        gsim_model_destroy(L.model);
        return hip_fail(e, "clear query");
    }
    // the host copies of the inputs are no longer needed
    for (std::vector<float>* v : {&q->mu, &q->lam, &q->ktri, &q->mass, &q->contact, &q->x0v0, &q->target})
        std::vector<float>().swap(*v);
    std::vector<Tile>().swap(q->tiles);
    L.q = std::move(q);
    L.t_admit = now_s();
    E->live.push_back(std::move(L));
    E->admitted++;
    return GSIM_OK;
}

void base_step(const Live& L, StepDev<float>& r) {
    std::memset(&r, 0, sizeof r);
    const QLayout& ly = L.q->lay;
    r.mu = L.q->ne ? L.F(ly.mu) : nullptr;
    r.lam = L.q->ne ? L.F(ly.lam) : nullptr;
    r.ktri = L.q->nt ? L.F(ly.ktri) : nullptr;
    r.mass = L.F(ly.mass);
    r.contact = L.F(ly.contact);
}

// Decides the next micro-step of a live query and fills its launch record.
int next_op(const Live& L, StepDev<float>& r) {
    const Query& q = *L.q;
    const QLayout& ly = q.lay;
    const int64_t S = 6 * q.np, np = q.np;
    base_step(L, r);
    if (L.phase == PH_FWD) {
        const int t = L.t;
        r.x = t == 0 ? L.F(ly.s0) : L.F((t - 1) & 1 ? ly.sB : ly.sA);
        r.v = r.x + 3 * np;
        r.x_abs = t == 0;  // the uploaded start state is absolute; later states are displacements
        r.xo = L.F(t & 1 ? ly.sB : ly.sA);
        r.vo = r.xo + 3 * np;
        if (t % q.K == 0) {
            r.ckx = L.F(ly.ckpt) + (int64_t)(t / q.K) * S;
            r.ckv = r.ckx + 3 * np;
        }
        return OP_FWD;
    }
    if (L.phase == PH_LOSS) {
        const int t = q.T - 1;
        r.x = L.F(t & 1 ? ly.sB : ly.sA);
        r.target = L.F(ly.target);
        r.loss = L.F(ly.loss);
        r.xbo = L.F(ly.seed);
        r.vbo = r.xbo + 3 * np;
        return OP_LOSS;
    }
    if (L.phase == PH_BWD) {
        const int t0 = L.seg * q.K, t1 = std::min(q.T, t0 + q.K), Ls = t1 - t0;
        const float* ck = L.F(ly.ckpt) + (int64_t)L.seg * S;
        float* sg = L.F(ly.seg);
        if (L.j + 1 < Ls) {  // recompute state t0 + j + 1
            r.x = L.j == 0 ? ck : sg + (int64_t)(L.j - 1) * S;
            r.v = r.x + 3 * np;
            r.xo = sg + (int64_t)L.j * S;
            r.vo = r.xo + 3 * np;
            return OP_FWD;
        }
        const int t = L.ta;
        r.x = t == t0 ? ck : sg + (int64_t)(t - t0 - 1) * S;
        r.v = r.x + 3 * np;
        r.xb = L.qa == 0 ? L.F(ly.seed) : L.F((L.qa - 1) & 1 ? ly.aB : ly.aA);
        r.vb = r.xb + 3 * np;
        r.xbo = L.F(L.qa & 1 ? ly.aB : ly.aA);
        r.vbo = r.xbo + 3 * np;
        // adjoint-force hand-off (as in the rollout backward): this step's particle pass
        // stores step t-1's adjoint force, the element pass of the next one reads it
        float* fbar = reinterpret_cast<float*>(L.model->ws + L.model->L.fbar);
        if (t > 0) r.fbo = fbar + (int64_t)(L.qa & 1) * 3 * np;
        if (L.qa > 0) r.fb = fbar + (int64_t)((L.qa - 1) & 1) * 3 * np;
        r.g_mu = q.ne ? L.F(ly.g_mu) : nullptr;
        r.g_lam = q.ne ? L.F(ly.g_lam) : nullptr;
        r.g_ktri = q.nt ? L.F(ly.g_ktri) : nullptr;
        r.g_mass = L.F(ly.g_mass);
        r.g_contact = L.F(ly.g_contact);
        return OP_ADJ;
    }
    r.g_contact = L.F(ly.g_contact);
    return OP_FIN;
}

void advance(Live& L, int op) {
    const Query& q = *L.q;
    if (op == OP_FWD && L.phase == PH_FWD) {
        if (++L.t == q.T) L.phase = PH_LOSS;
        return;
    }
    if (op == OP_LOSS) {
        L.phase = PH_BWD;
        L.seg = (q.T + q.K - 1) / q.K - 1;
        L.j = 0;
        L.ta = q.T - 1;
        L.qa = 0;
        return;
    }
    if (op == OP_FWD) {  // recompute
        L.j++;
        return;
    }
    if (op == OP_ADJ) {
        L.qa++;
        const int t0 = L.seg * q.K;
        if (L.ta == t0) {
            if (L.seg == 0) {
                L.phase = PH_FIN;
                return;
            }
            L.seg--;
            L.j = 0;
        }
        L.ta--;
    }
}

// Hands a retired query's results from the ring to the caller's buffers.
void deliver(gsim_engine* E, Pending& P) {
    const Query& q = *P.q;
    const QLayout& ly = q.lay;
    const char* r = E->results.host + P.off;
    auto out = [&](float* dst, size_t o, int64_t n) {
        if (dst && n) std::memcpy(dst, r + (o - ly.g_mu), (size_t)n * 4);
    };
    out(q.o_mu, ly.g_mu, q.ne);
    out(q.o_lam, ly.g_lam, q.ne);
    out(q.o_ktri, ly.g_ktri, q.nt);
    out(q.o_mass, ly.g_mass, q.np);
    out(q.o_contact, ly.g_contact, 4);
    float loss;
    int32_t flags[2];
    std::memcpy(&loss, r + (ly.loss - ly.g_mu), 4);
    std::memcpy(flags, E->results.host + P.flags_at, sizeof flags);
    E->done.push_back({q.id, loss, q.t_submit, P.t_admit, now_s(), flags[0] ? GSIM_E_NONFINITE : GSIM_OK});
    E->completed++;
}

// Delivers the finished queries whose copies have completed (all of them, waiting,
// when `wait`), oldest first.
int retire(gsim_engine* E, bool wait) {
    ResultRing& R = E->results;
    while (!R.q.empty()) {
        Pending& P = R.q.front();
        if (!P.evt) break;  // its round has not recorded its event yet
        if (wait) {
            HIP_TRY(hipEventSynchronize(P.evt), "wait for results");
        } else {
            const hipError_t e = hipEventQuery(P.evt);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return hip_fail(e, "query results");
        }
        deliver(E, P);
        hipEvent_t ev = P.evt;
        R.q.pop_front();
        if (R.q.empty() || R.q.front().evt != ev) R.free_events.push_back(ev);
    }
    return GSIM_OK;
}

int finish(gsim_engine* E, Live& L) {
    Query& q = *L.q;
    const QLayout& ly = q.lay;
    hipStream_t s = E->stream;
    // asynchronous: the gradient block and the status words go to the pinned ring and
    // reach the caller when the round's event has completed
    const size_t span = ly.loss + 4 - ly.g_mu, need = (span + 15) / 16 * 16 + 16;
    ResultRing& R = E->results;
    size_t off = 0;
    bool placed = R.place(need, off);
    while (!placed && !R.q.empty() && R.q.front().evt) {  // make room: wait for the oldest
        Pending& P = R.q.front();
        HIP_TRY(hipEventSynchronize(P.evt), "wait for results");
        deliver(E, P);
        hipEvent_t ev = P.evt;
        R.q.pop_front();
        if (R.q.empty() || R.q.front().evt != ev) R.free_events.push_back(ev);
        placed = R.place(need, off);
    }
    if (placed) {
        Pending P;
        P.off = off;
        P.bytes = need;
        P.flags_at = off + (span + 15) / 16 * 16;
        P.t_admit = L.t_admit;
        HIP_TRY(hipMemcpyAsync(R.host + off, L.base + ly.g_mu, span, hipMemcpyDeviceToHost, s), "copy out");
        HIP_TRY(hipMemcpyAsync(R.host + P.flags_at, L.model->ws + L.model->L.bflag, 8, hipMemcpyDeviceToHost, s),
                "copy out");
        P.q = std::move(L.q);
        R.q.push_back(std::move(P));
        E->round_finished = true;
        gsim_model_destroy(L.model);
        E->pool.release(L.off, R.q.back().q->lay.total);  // later users of the region come after the copies
        return GSIM_OK;
    }
    // (results larger than the ring, or the ring held by this round alone: copy and wait)
    float loss = 0.f;
    int32_t flags[2] = {0, 0};
    auto down = [&](float* dst, size_t o, int64_t n) -> hipError_t {
        if (!dst || n == 0) return hipSuccess;
        return hipMemcpyAsync(dst, L.base + o, n * 4, hipMemcpyDeviceToHost, s);
    };
    HIP_TRY(down(&loss, ly.loss, 1), "copy out");
    HIP_TRY(down(q.o_mu, ly.g_mu, q.ne), "copy out");
    HIP_TRY(down(q.o_lam, ly.g_lam, q.ne), "copy out");
    HIP_TRY(down(q.o_ktri, ly.g_ktri, q.nt), "copy out");
    HIP_TRY(down(q.o_mass, ly.g_mass, q.np), "copy out");
    HIP_TRY(down(q.o_contact, ly.g_contact, 4), "copy out");
    // the query's status words (its model's first body) come out with its results
    HIP_TRY(hipMemcpyAsync(flags, L.model->ws + L.model->L.bflag, sizeof flags, hipMemcpyDeviceToHost, s), "copy out");
    HIP_TRY(hipStreamSynchronize(s), "copy out");
    E->done.push_back({q.id, loss, q.t_submit, L.t_admit, now_s(), flags[0] ? GSIM_E_NONFINITE : GSIM_OK});
    gsim_model_destroy(L.model);
    E->pool.release(L.off, q.lay.total);
    E->completed++;
    return GSIM_OK;
}

// One micro-step of every live query: plan each query's next operation, upload the
// round's tables in one copy, run the singular launches (loss seeds, final
// reductions), then one element launch and one particle launch over the forward and
// the adjoint tiles of every query together; finally advance the queries and finish
// the completed ones.
int micro_round(gsim_engine* E) {
    const int n = (int)E->live.size();
    E->ticks++;
    E->live_sum += n;
    std::vector<int> ops(n);
    std::vector<StepDev<float>> sd(n);
    for (int i = 0; i < n; ++i) ops[i] = next_op(E->live[i], sd[i]);
    // segment tables: each query with a forward or adjoint micro-step contributes its
    // resident element tiles and particle tiles; each workgroup of the round's two
    // launches finds its tile in them (XCD order over the concatenation)
    std::vector<TileSeg> seg[2];  // element pass, particle pass
    int total[2] = {0, 0};
    for (int i = 0; i < n; ++i) {
        if (ops[i] != OP_FWD && ops[i] != OP_ADJ) continue;
        const Live& L = E->live[i];
        const Tile* t = reinterpret_cast<const Tile*>(L.base + L.q->lay.tiles);
        const int32_t flags = ops[i] == OP_ADJ ? TILE_ADJ : 0;
        const int cnt[2] = {L.q->n_etiles, L.q->n_ptiles};
        for (int k = 0; k < 2; ++k) {
            if (cnt[k] == 0) continue;
            seg[k].push_back({k == 0 ? t : t + L.q->n_etiles, total[k], cnt[k], i, flags});
            total[k] += cnt[k];
        }
    }
    int grid[2];
    for (int k = 0; k < 2; ++k)
        grid[k] = total[k] < N_XCD ? total[k] : (total[k] + N_XCD - 1) / N_XCD * N_XCD;
    if (grid[0] > E->max_tiles || grid[1] > E->max_tiles)
        return fail(GSIM_E_WORKSPACE, "a round needs %d / %d tiles, the engine holds %lld", grid[0], grid[1],
                    (long long)E->max_tiles);
    // one upload: [ModelDev x n][StepDev x n][element segments][particle segments]
    const size_t md_sz = sizeof(ModelDev<float>), sd_sz = sizeof(StepDev<float>);
    const size_t o_md = 0, o_sd = aup(md_sz * n), o_s0 = aup(o_sd + sd_sz * n);
    const size_t o_s1 = aup(o_s0 + sizeof(TileSeg) * seg[0].size());
    const size_t o = aup(o_s1 + sizeof(TileSeg) * seg[1].size());
    if (o > E->head_bytes) return fail(GSIM_E_WORKSPACE, "round tables exceed the engine's table capacity");
    const int r = E->ring;
    E->ring = (E->ring + 1) % RING;
    HIP_TRY(hipEventSynchronize(E->blob_evt[r]), "wait for table ring");
    char* h = E->blob_host[r];
    for (int i = 0; i < n; ++i) std::memcpy(h + o_md + i * md_sz, E->live[i].model->md_host.data(), md_sz);
    std::memcpy(h + o_sd, sd.data(), sd_sz * n);
    std::memcpy(h + o_s0, seg[0].data(), sizeof(TileSeg) * seg[0].size());
    std::memcpy(h + o_s1, seg[1].data(), sizeof(TileSeg) * seg[1].size());
    char* d = E->blob_dev[r];
    HIP_TRY(hipMemcpyAsync(d, h, o, hipMemcpyHostToDevice, E->stream), "upload tick tables");
    const ModelDev<float>* dmd = reinterpret_cast<const ModelDev<float>*>(d + o_md);
    const StepDev<float>* dsd = reinterpret_cast<const StepDev<float>*>(d + o_sd);
    const int dummy_row = E->live[0].model->n_ptile_rows;  // empty tiles reduce into model 0's spare row
    // per-query singular launches (loss seed, contact reduction)
    for (int i = 0; i < n; ++i) {
        gsim_model* m = E->live[i].model;
        const ModelDev<float>* own = reinterpret_cast<const ModelDev<float>*>(m->ws + m->L.model);
        const Tile* own_pt = reinterpret_cast<const Tile*>(m->ws + m->L.ptiles);
        if (ops[i] == OP_LOSS)
            LAUNCH_TRY(launch_loss<float>(own, dsd + i, own_pt, m->n_ptiles, m->pblock, m->pitems, 1, E->stream), "loss");
        if (ops[i] == OP_FIN) LAUNCH_TRY(launch_contact_reduce<float>(own, dsd + i, 1, E->stream), "contact reduce");
    }
    // the element launch and the particle launch over every query's tiles (element LDS:
    // the largest tile among the queries in this round, forward or adjoint)
    const int block = 256;
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const gsim_model* m = E->live[i].model;
        if (ops[i] == OP_FWD) lds = std::max(lds, (size_t)m->etile_words[0] * sizeof(float));
        if (ops[i] == OP_ADJ) lds = std::max(lds, (size_t)m->etile_words[1] * sizeof(float));
    }
    LAUNCH_TRY(launch_mixed<float>(dmd, dsd, reinterpret_cast<const TileSeg*>(d + o_s0), (int)seg[0].size(), total[0],
                                   grid[0], reinterpret_cast<const TileSeg*>(d + o_s1), (int)seg[1].size(), total[1],
                                   grid[1], dummy_row, block, lds, E->stream),
               "element and particle passes");
    HIP_TRY(hipEventRecord(E->blob_evt[r], E->stream), "record tick");
    // advance; finish completed queries
    std::vector<Live> keep;
    keep.reserve(n);
    E->round_finished = false;
    for (int i = 0; i < n; ++i) {
        Live& L = E->live[i];
        if (ops[i] == OP_FIN) {
            int rc = finish(E, L);
            if (rc) return rc;
            continue;
        }
        advance(L, ops[i]);
        keep.push_back(std::move(L));
    }
    E->live.swap(keep);
    if (E->round_finished) {  // one event for the result copies of this round
        ResultRing& R = E->results;
        hipEvent_t ev = nullptr;
        if (!R.free_events.empty()) {
            ev = R.free_events.back();
            R.free_events.pop_back();
        } else {
            HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "result event");
        }
        HIP_TRY(hipEventRecord(ev, E->stream), "record results");
        for (auto it = R.q.rbegin(); it != R.q.rend() && !it->evt; ++it) it->evt = ev;
    }
    return GSIM_OK;
}

int tick(gsim_engine* E, int* n_live, int* n_queued) {
    if (int rc = retire(E, false)) return rc;
    // 1. admission, FIFO while the head fits; the admitted queries' set-up copies move
    // in one staged batch
    while (!E->queue.empty() && (int)E->live.size() < E->max_live) {
        size_t off;
        if (!E->pool.alloc(E->queue.front()->lay.total, off)) break;
        std::unique_ptr<Query> q = std::move(E->queue.front());
        E->queue.pop_front();
        int rc = admit(E, q, off);
        if (rc) {
            (void)E->stage.flush();  // what was staged for the region lands before it is reused
            E->pool.release(off, q ? q->lay.total : 0);
            return rc;
        }
    }
    HIP_TRY(E->stage.flush(), "stage queries");
    // 2. micro-step rounds
    for (int k = 0; k < E->micro_per_tick && !E->live.empty(); ++k)
        if (int rc = micro_round(E)) return rc;
    // 3. results: those ready now; all of them once nothing is live or queued, so that
    // an idle engine has delivered every answer
    if (int rc = retire(E, E->live.empty() && E->queue.empty())) return rc;
    if (n_live) *n_live = (int)E->live.size();
    if (n_queued) *n_queued = (int)E->queue.size();
    return GSIM_OK;
}

}  // namespace

extern "C" {

int gsim_engine_create(void* d_pool, size_t pool_bytes, int max_live, int64_t max_tiles, void* stream,
                       gsim_engine** out) {
    if (!d_pool || !out || max_live < 1 || max_tiles < 64) return fail(GSIM_E_INVALID, "bad engine arguments");
    if (((uintptr_t)d_pool & 255) != 0) return fail(GSIM_E_INVALID, "pool must be 256-byte aligned");
    gsim_engine* E = new (std::nothrow) gsim_engine();
    if (!E) return fail(GSIM_E_INVALID, "out of host memory");
    E->pool_base = (char*)d_pool;
    E->max_live = max_live;
    E->max_tiles = max_tiles;
    E->stream = (hipStream_t)stream;
    // a ring slot: the round's uploaded tables (models, steps, segment tables)
    E->head_bytes = aup((sizeof(ModelDev<float>) + sizeof(StepDev<float>) + 2 * sizeof(TileSeg)) * max_live + 4 * 256);
    E->blob_bytes = E->head_bytes;
    if ((size_t)RING * E->blob_bytes >= pool_bytes) {
        delete E;
        return fail(GSIM_E_WORKSPACE, "pool too small for the engine's tables");
    }
    for (int r = 0; r < RING; ++r) {
        E->blob_dev[r] = E->pool_base + r * E->blob_bytes;
        hipError_t e = hipHostMalloc((void**)&E->blob_host[r], E->head_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&E->blob_evt[r], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(E->blob_evt[r], E->stream);
        if (e != hipSuccess) {
            gsim_engine_destroy(E);
            return hip_fail(e, "engine tables");
        }
    }
    // staging chunks (device mirrors after the table ring) and the pinned result ring
    Stager& st = E->stage;
    st.cap = STAGE_CHUNK_BYTES;
    st.stream = E->stream;
    size_t used = RING * E->blob_bytes;
    if (used + Stager::N * st.cap >= pool_bytes) {
        gsim_engine_destroy(E);
        return fail(GSIM_E_WORKSPACE, "pool too small for the engine's tables and staging");
    }
    for (int c = 0; c < Stager::N; ++c) {
        st.dev[c] = E->pool_base + used + c * st.cap;
        hipError_t e = hipHostMalloc((void**)&st.host[c], st.cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&st.evt[c], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(st.evt[c], E->stream);
        if (e != hipSuccess) {
            gsim_engine_destroy(E);
            return hip_fail(e, "engine staging");
        }
    }
    used += Stager::N * st.cap;
    E->results.cap = RESULT_RING_BYTES;
    if (hipError_t e = hipHostMalloc((void**)&E->results.host, E->results.cap, hipHostMallocDefault)) {
        gsim_engine_destroy(E);
        return hip_fail(e, "engine result ring");
    }
    E->pool.init(pool_bytes - used);
    E->pool_base += used;
    E->store_limit = E->pool.size / 64;
    *out = E;
    return GSIM_OK;
}

int gsim_engine_destroy(gsim_engine* E) {
    if (!E) return GSIM_OK;
    (void)hipStreamSynchronize(E->stream);
    for (Live& L : E->live) gsim_model_destroy(L.model);
    for (int r = 0; r < RING; ++r) {
        if (E->blob_evt[r]) (void)hipEventDestroy(E->blob_evt[r]);
        if (E->blob_host[r]) (void)hipHostFree(E->blob_host[r]);
    }
    for (int c = 0; c < Stager::N; ++c) {
        if (E->stage.evt[c]) (void)hipEventDestroy(E->stage.evt[c]);
        if (E->stage.host[c]) (void)hipHostFree(E->stage.host[c]);
    }
    std::vector<hipEvent_t> evs = E->results.free_events;
    for (const Pending& P : E->results.q)
        if (P.evt && (evs.empty() || evs.back() != P.evt)) evs.push_back(P.evt);
    std::sort(evs.begin(), evs.end());
    evs.erase(std::unique(evs.begin(), evs.end()), evs.end());
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    if (E->results.host) (void)hipHostFree(E->results.host);
    delete E;
    return GSIM_OK;
}

int gsim_engine_query_bytes(const gsim_query* q, size_t* bytes) {
    if (!q || !q->desc || !bytes) return fail(GSIM_E_INVALID, "NULL argument");
    gsim_plan* P = nullptr;
    int rc = plan_create(q->desc, &P, false);  // queries run the two-pass path only
    if (rc) return rc;
    *bytes = qlayout(P, q->n_steps, q->ckpt_every).total;
    gsim_plan_destroy(P);
    return GSIM_OK;
}

int gsim_engine_prepare(const gsim_query* in, gsim_prepared** out) {
    if (!in || !in->desc || !out) return fail(GSIM_E_INVALID, "NULL argument");
    *out = nullptr;
    const double t_arrive = now_s();
    const gsim_model_desc* d = in->desc;
    if (d->dtype != GSIM_F32 || d->n_bodies != 1) return fail(GSIM_E_UNSUPPORTED, "queries are single FP32 bodies");
    if (d->air_on && d->air_on[0]) return fail(GSIM_E_UNSUPPORTED, "queries do not model lift/drag");
    if (in->n_steps < 1 || in->ckpt_every < 1) return fail(GSIM_E_INVALID, "n_steps and ckpt_every must be >= 1");
    if (!in->mass || !in->contact || !in->x0 || !in->v0 || !in->target) return fail(GSIM_E_INVALID, "NULL input");
    if (d->n_tets && (!in->mu || !in->lam)) return fail(GSIM_E_INVALID, "mu and lam are required");
    if (d->n_tris && !in->k_tri) return fail(GSIM_E_INVALID, "k_tri is required");
    // parameters are on the host here: a query that could only produce non-finite
    // results is refused before it takes a slot
    auto positive = [](const float* a, int64_t n, const char* what) -> int {
        for (int64_t i = 0; i < n; ++i) {
            if (!std::isfinite(a[i])) return fail(GSIM_E_NONFINITE, "%s[%lld] is not finite", what, (long long)i);
            if (!(a[i] > 0.f)) return fail(GSIM_E_INVALID, "%s[%lld] must be > 0", what, (long long)i);
        }
        return GSIM_OK;
    };
    auto finite = [](const float* a, int64_t n, const char* what) -> int {
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(a[i])) return fail(GSIM_E_NONFINITE, "%s[%lld] is not finite", what, (long long)i);
        return GSIM_OK;
    };
    if (int rc = positive(in->mass, d->n_particles, "mass")) return rc;
    if (d->n_tets)
        if (int rc = positive(in->mu, d->n_tets, "mu")) return rc;
    if (d->n_tets)
        if (int rc = positive(in->lam, d->n_tets, "lam")) return rc;
    if (d->n_tris)
        if (int rc = positive(in->k_tri, d->n_tris, "k_tri")) return rc;
    if (int rc = finite(in->contact, 4, "contact")) return rc;
    for (int k = 0; k < 4; ++k)
        if (in->contact[k] < 0.f) return fail(GSIM_E_INVALID, "contact[%d] must be >= 0", k);
    if (int rc = finite(in->x0, 3 * d->n_particles, "x0")) return rc;
    if (int rc = finite(in->v0, 3 * d->n_particles, "v0")) return rc;
    if (int rc = finite(in->target, 3 * d->n_particles, "target")) return rc;
    try {
        std::unique_ptr<Query> q(new Query());
        gsim_plan* P = nullptr;
        int rc = plan_create(d, &P, false);
        if (rc) return rc;
        q->plan.reset(P);
        q->T = in->n_steps;
        q->K = in->ckpt_every;
        q->np = P->np;
        q->ne = P->ne;
        q->nt = P->nt;
        q->lay = qlayout(P, q->T, q->K);
        auto cp = [](std::vector<float>& v, const float* src, int64_t n) { v.assign(src, src + n); };
        if (q->ne) {
            cp(q->mu, in->mu, q->ne);
            cp(q->lam, in->lam, q->ne);
        }
        if (q->nt) cp(q->ktri, in->k_tri, q->nt);
        cp(q->mass, in->mass, q->np);
        cp(q->contact, in->contact, 4);
        q->x0v0.resize(6 * q->np);
        std::memcpy(q->x0v0.data(), in->x0, 12 * q->np);
        std::memcpy(q->x0v0.data() + 3 * q->np, in->v0, 12 * q->np);
        cp(q->target, in->target, 3 * q->np);
        q->o_mu = in->out_mu;
        q->o_lam = in->out_lam;
        q->o_ktri = in->out_k_tri;
        q->o_mass = in->out_mass;
        q->o_contact = in->out_contact;
        q->t_submit = t_arrive;
        *out = reinterpret_cast<gsim_prepared*>(q.release());
    } catch (const std::bad_alloc&) {
        return fail(GSIM_E_INVALID, "out of host memory");
    }
    return GSIM_OK;
}

int gsim_engine_submit_prepared(gsim_engine* E, gsim_prepared* prep, int64_t* id) {
    if (!E || !prep) return fail(GSIM_E_INVALID, "NULL argument");
    std::unique_ptr<Query> q(reinterpret_cast<Query*>(prep));  // owned from here on, queued or not
    try {
        if (q->K > 1 && E->store_limit > 0) {  // every state stored when it fits the limit
            const QLayout all = qlayout(q->plan.get(), q->T, 1);
            if (all.total <= E->store_limit) {
                q->K = 1;
                q->lay = all;
            }
        }
        if (q->lay.total > E->pool.size)
            return fail(GSIM_E_WORKSPACE, "query needs %zu bytes, the pool has %zu", q->lay.total, E->pool.size);
        q->id = E->next_id++;
        if (id) *id = q->id;
        E->queue.push_back(std::move(q));
    } catch (const std::bad_alloc&) {
        return fail(GSIM_E_INVALID, "out of host memory");
    }
    return GSIM_OK;
}

int gsim_prepared_destroy(gsim_prepared* prep) {
    delete reinterpret_cast<Query*>(prep);
    return GSIM_OK;
}

int gsim_engine_submit(gsim_engine* E, const gsim_query* in, int64_t* id) {
    if (!E) return fail(GSIM_E_INVALID, "NULL engine");
    gsim_prepared* prep = nullptr;
    if (int rc = gsim_engine_prepare(in, &prep)) return rc;
    return gsim_engine_submit_prepared(E, prep, id);
}

int gsim_engine_tick(gsim_engine* E, int* n_live, int* n_queued) {
    if (!E) return fail(GSIM_E_INVALID, "NULL engine");
    try {
        return tick(E, n_live, n_queued);
    } catch (const std::bad_alloc&) {
        return fail(GSIM_E_INVALID, "out of host memory");
    }
}

int gsim_engine_poll(gsim_engine* E, gsim_result* out, int max, int* n) {
    if (!E || !n) return fail(GSIM_E_INVALID, "NULL argument");
    int k = 0;
    while (k < max && !E->done.empty()) {
        const Done& d = E->done.front();
        out[k].id = d.id;
        out[k].loss = d.loss;
        out[k].t_submit = d.t_submit;
        out[k].t_admit = d.t_admit;
        out[k].t_done = d.t_done;
        out[k].status = d.status;
        E->done.erase(E->done.begin());
        ++k;
    }
    *n = k;
    return GSIM_OK;
}

int gsim_engine_set_micro_steps(gsim_engine* E, int rounds) {
    if (!E) return fail(GSIM_E_INVALID, "NULL engine");
    if (rounds < 1 || rounds > 256) return fail(GSIM_E_INVALID, "micro-step rounds per tick must be in [1, 256]");
    E->micro_per_tick = rounds;
    return GSIM_OK;
}

int gsim_engine_set_store_limit(gsim_engine* E, size_t bytes) {
    if (!E) return fail(GSIM_E_INVALID, "NULL engine");
    E->store_limit = bytes;
    return GSIM_OK;
}

int gsim_engine_stats(const gsim_engine* E, int64_t* ticks, int64_t* admitted, int64_t* completed,
                      double* mean_live, size_t* pool_free) {
    if (!E) return fail(GSIM_E_INVALID, "NULL engine");
    if (ticks) *ticks = E->ticks;
    if (admitted) *admitted = E->admitted;
    if (completed) *completed = E->completed;
    if (mean_live) *mean_live = E->ticks ? E->live_sum / E->ticks : 0.0;
    if (pool_free) *pool_free = E->pool.free_bytes();
    return GSIM_OK;
}

}  // extern "C"

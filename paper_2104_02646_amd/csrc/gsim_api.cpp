// Host runtime and C-ABI of libgsim (declared in include/gsim.h).
//
// Planning (host, once per model): validation of the description, tet
// orientation, rest-shape precompute (Dm^-1, volume / area, rest dihedral
// angle), the deterministic gather table (each particle's element corners in a
// fixed order), and workgroup tiles.  Device memory is caller-owned: the model
// carves its records, buffers and launch tables out of one workspace.
//
// Every step launches an element pass and a particle pass (forward or adjoint).
// The per-launch pointers live in StepDev records in the workspace; a call
// builds its records on the host, uploads only what changed, and replays its
// launch sequence -- as plain launches or as a captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "gsim_host.h"

using namespace gsim;

namespace {
thread_local std::string g_err;
}  // namespace

namespace gsim {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(GSIM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

void xcd_order(const std::vector<Tile>& nat, int empty_kind, int dummy_id, std::vector<Tile>& out, int& grid) {
    const int64_t N = (int64_t)nat.size();
    if (N < N_XCD) {
        out = nat;
        grid = (int)N;
        return;
    }
    const int64_t G = (N + N_XCD - 1) / N_XCD;
    grid = (int)(G * N_XCD);
    Tile empty{};
    empty.kind = empty_kind;
    empty.count = 0;
    empty.id = dummy_id;
    out.assign(grid, empty);
    for (int64_t t = 0; t < N; ++t) out[(t % G) * N_XCD + t / G] = nat[t];
}

}  // namespace gsim

namespace {

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

#define LAUNCH_TRY(call, what)                                            \
    do {                                                                  \
        int rc_ = (call);                                                 \
        if (rc_) return hip_fail((hipError_t)rc_, what);                  \
    } while (0)

struct D3 {
    double x, y, z;
};
D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
D3 crs(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double dt3(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
double nrm(D3 a) { return std::sqrt(dt3(a, a)); }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace


namespace {

bool finite(double v) { return std::isfinite(v); }

int check_offsets(const int64_t* off, int nb, int64_t total, const char* name) {
    if (total == 0 && off == nullptr) return GSIM_OK;
    if (!off) return fail(GSIM_E_INVALID, "%s offsets are NULL but the count is %lld", name, (long long)total);
    if (off[0] != 0 || off[nb] != total)
        return fail(GSIM_E_INVALID, "%s offsets must start at 0 and end at %lld", name, (long long)total);
    for (int b = 0; b < nb; ++b)
        if (off[b + 1] < off[b]) return fail(GSIM_E_INVALID, "%s offsets decrease at body %d", name, b);
    return GSIM_OK;
}

// Rest dihedral angle with the same orientation convention as the kernels.
double rest_angle(const D3 x[4]) {
    D3 E = sub(x[3], x[2]);
    D3 N1 = crs(sub(x[0], x[2]), sub(x[0], x[3]));
    D3 N2 = crs(sub(x[1], x[3]), sub(x[1], x[2]));
    double el = nrm(E);
    return std::atan2(-dt3(crs(N1, N2), E) / el, dt3(N1, N2));
}

// Greedy colouring for the fused path: per body and element kind, each element
// (in index order) takes the smallest colour none of its particles has seen yet.
// Elements are then listed by (colour, index) with colour boundaries in coff.
void colour_elements(gsim_plan* P) {
    const int nb = P->nb;
    P->ftet.assign(P->ne, 0);
    P->ftri.assign(P->nt, 0);
    P->fhin.assign(P->nh, 0);
    P->coff.clear();
    P->cbase.assign(3 * nb, 0);
    P->ncol.assign(3 * nb, 0);
    P->fused_ok = true;
    P->coloured = true;
    std::vector<uint64_t> used_lo, used_hi;
    for (int b = 0; b < nb; ++b) {
        const int64_t p0 = P->poff[b], npb = P->poff[b + 1] - p0;
        for (int kind = 0; kind < 3; ++kind) {
            const std::vector<int64_t>& off = kind == 0 ? P->eoff : kind == 1 ? P->toff : P->hoff;
            const std::vector<int32_t>& idx = kind == 0 ? P->tet_idx : kind == 1 ? P->tri_idx : P->hin_idx;
            std::vector<int32_t>& ford = kind == 0 ? P->ftet : kind == 1 ? P->ftri : P->fhin;
            const int64_t n = kind == 0 ? P->ne : kind == 1 ? P->nt : P->nh;
            const int nc = kind == 1 ? 3 : 4;
            const int64_t e0 = off[b], e1 = off[b + 1];
            used_lo.assign(npb, 0);
            used_hi.assign(npb, 0);
            std::vector<int> col(e1 - e0, 0);
            int ncolours = 0;
            for (int64_t e = e0; e < e1; ++e) {
                uint64_t lo = 0, hi = 0;
                for (int c = 0; c < nc; ++c) {
                    const int64_t li = idx[c * n + e] - p0;
                    lo |= used_lo[li];
                    hi |= used_hi[li];
                }
                int k = -1;
                if (~lo) k = __builtin_ctzll(~lo);
                else if (~hi) k = 64 + __builtin_ctzll(~hi);
                if (k < 0) {
                    P->fused_ok = false;
                    k = 0;
                }
                col[e - e0] = k;
                ncolours = std::max(ncolours, k + 1);
                for (int c = 0; c < nc; ++c) {
                    const int64_t li = idx[c * n + e] - p0;
                    if (k < 64) used_lo[li] |= 1ull << k;
                    else used_hi[li] |= 1ull << (k - 64);
                }
            }
            // counting sort by colour (stable: index order inside a colour)
            std::vector<int64_t> start(ncolours + 1, 0);
            for (int64_t e = e0; e < e1; ++e) start[col[e - e0] + 1]++;
            for (int k = 0; k < ncolours; ++k) start[k + 1] += start[k];
            P->cbase[3 * b + kind] = (int32_t)P->coff.size();
            P->ncol[3 * b + kind] = ncolours;
            for (int k = 0; k <= ncolours; ++k) P->coff.push_back((int32_t)(e0 + start[k]));
            std::vector<int64_t> pos(start.begin(), start.end() - 1);
            for (int64_t e = e0; e < e1; ++e) ford[e0 + pos[col[e - e0]]++] = (int32_t)e;
        }
    }
}

// Element tiles of the two-pass path.  Per body and element kind, consecutive
// elements are cut into tiles of at most tile_elems elements, a tile ending early when
// its adjoint LDS (8 words per tile particle, 4 per corner) would exceed
// ETILE_WORDS.  Per tile: its particles in increasing index order (the tile
// particles); its corners ordered by (tile particle, element, corner), so each
// tile particle's corners form one contiguous run; corner code = tile-local
// particle | position in that order << 16.  The kernels sum each run into one
// partial per (tile, particle).  Partials are stored sliced-ELL: each body's
// particles are cut into slices of 64 from the body's first particle; slice g
// holds width_g = max partials per particle of its particles, and the k-th tile
// (plan order) touching the particle at lane j writes slot gbase[g] + 64 k + j.
// Everything here depends only on the body itself, never on the rest of a batch.
int build_tiles(gsim_plan* P) {
    const int nb = P->nb;
    P->etiles.clear();
    P->tp_id.clear();
    P->tp_run.clear();
    P->tet_code.assign(4 * P->ne, 0);
    P->tri_code.assign(3 * P->nt, 0);
    P->hin_code.assign(4 * P->nh, 0);
    P->etile_words[0] = P->etile_words[1] = 0;
    std::vector<int32_t> mark(P->np, -1), loc(P->np, 0), parts, cnt, fill;
    for (int b = 0; b < nb; ++b)
        for (int kind = 0; kind < 3; ++kind) {
            const std::vector<int64_t>& off = kind == 0 ? P->eoff : kind == 1 ? P->toff : P->hoff;
            const std::vector<int32_t>& idx = kind == 0 ? P->tet_idx : kind == 1 ? P->tri_idx : P->hin_idx;
            std::vector<uint32_t>& code = kind == 0 ? P->tet_code : kind == 1 ? P->tri_code : P->hin_code;
            const int64_t n = kind == 0 ? P->ne : kind == 1 ? P->nt : P->nh;
            const int nc = kind == 1 ? 3 : 4;
            // LDS words of the adjoint per tile particle and per corner (triangles with
            // air also stage velocities and keep a velocity adjoint per corner)
            const bool air = kind == 1 && P->air_on[b];
            const int64_t wp = air ? 12 : 8, wc = air ? 8 : 4;
            int64_t e = off[b];
            while (e < off[b + 1]) {
                const int32_t tile = (int32_t)P->etiles.size();
                const int64_t s = e;
                parts.clear();
                while (e < off[b + 1] && e - s < P->tile_elems) {
                    int add = 0;
                    for (int c = 0; c < nc; ++c) add += mark[idx[c * n + e]] != tile;
                    const int64_t words = wp * (int64_t)(parts.size() + add) + wc * (int64_t)nc * (e - s + 1);
                    if (e > s && words > ETILE_WORDS) break;
                    for (int c = 0; c < nc; ++c) {
                        const int32_t p = idx[c * n + e];
                        if (mark[p] != tile) {
                            mark[p] = tile;
                            parts.push_back(p);
                        }
                    }
                    ++e;
                }
                // increasing index order: a scan of the marks over the tile's index range
                // when that range is narrow (tiles are spatially local), else a sort
                {
                    int32_t lo = INT32_MAX, hi = -1;
                    for (int32_t p : parts) {
                        lo = std::min(lo, p);
                        hi = std::max(hi, p);
                    }
                    if (!parts.empty() && (int64_t)hi - lo < 8 * (int64_t)parts.size()) {
                        size_t k = 0;
                        for (int32_t p = lo; p <= hi; ++p)
                            if (mark[p] == tile) parts[k++] = p;
                    } else {
                        std::sort(parts.begin(), parts.end());
                    }
                }
                const int m = (int)parts.size();
                for (int j = 0; j < m; ++j) loc[parts[j]] = j;
                cnt.assign(m, 0);
                for (int64_t l = s; l < e; ++l)
                    for (int c = 0; c < nc; ++c) cnt[loc[idx[c * n + l]]]++;
                fill.assign(m, 0);
                for (int j = 1; j < m; ++j) fill[j] = fill[j - 1] + cnt[j - 1];
                for (int j = 0; j < m; ++j) P->tp_run.push_back(fill[j] | (cnt[j] << 16));
                for (int64_t l = s; l < e; ++l)
                    for (int c = 0; c < nc; ++c) {
                        const int j = loc[idx[c * n + l]];
                        code[c * n + l] = (uint32_t)j | ((uint32_t)fill[j]++ << 16);
                    }
                Tile t{};
                t.model = 0;
                t.body = b;
                t.kind = kind == 0 ? TILE_TET : kind == 1 ? TILE_TRI : TILE_HINGE;
                t.count = (int32_t)(e - s);
                t.begin = s;
                t.id = (int32_t)P->tp_id.size();
                t.pad = m;
                P->etiles.push_back(t);
                P->tp_id.insert(P->tp_id.end(), parts.begin(), parts.end());
                const int64_t corners = (int64_t)nc * (e - s);
                P->etile_words[0] = std::max<int64_t>(P->etile_words[0], (air ? 8 : 4) * (int64_t)m + 4 * corners);
                P->etile_words[1] = std::max<int64_t>(P->etile_words[1], wp * (int64_t)m + wc * corners);
                if ((int64_t)P->tp_id.size() > INT32_MAX) return fail(GSIM_E_UNSUPPORTED, "too many tile particles");
            }
        }
    // partial slots (sliced ELL)
    P->pdeg.assign(P->np, 0);
    for (int32_t p : P->tp_id) P->pdeg[p]++;
    P->gbase.clear();
    P->body_g0.assign(nb, 0);
    std::vector<int64_t> pbase(P->np);  // slot of partial 0 of each particle
    int64_t total = 0;
    for (int b = 0; b < nb; ++b) {
        P->body_g0[b] = (int32_t)P->gbase.size();
        for (int64_t s0 = P->poff[b]; s0 < P->poff[b + 1]; s0 += 64) {
            const int64_t s1 = std::min<int64_t>(s0 + 64, P->poff[b + 1]);
            int32_t w = 0;
            for (int64_t i = s0; i < s1; ++i) w = std::max(w, P->pdeg[i]);
            if (total + 64 * (int64_t)w > INT32_MAX) return fail(GSIM_E_UNSUPPORTED, "partial table exceeds 32-bit slots");
            P->gbase.push_back((int32_t)total);
            for (int64_t i = s0; i < s1; ++i) pbase[i] = total + (i - s0);
            total += 64 * (int64_t)w;
        }
    }
    P->nslot = total;
    std::vector<int32_t> cur(P->np, 0);
    P->tp_slot.resize(P->tp_id.size());
    for (size_t i = 0; i < P->tp_id.size(); ++i) {
        const int32_t p = P->tp_id[i];
        P->tp_slot[i] = (int32_t)(pbase[p] + 64 * (int64_t)cur[p]++);
    }
    return GSIM_OK;
}

// The corners of an element are distinct particles (the fused kernels update an
// element's corners in LDS with all reads before all writes).
bool distinct(const int32_t* id, int n) {
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (id[i] == id[j]) return false;
    return true;
}

int build_plan(const gsim_model_desc* d, gsim_plan* P, bool fused) {
    if (!d) return fail(GSIM_E_INVALID, "NULL description");
    if (d->dtype != GSIM_F32 && d->dtype != GSIM_F64) return fail(GSIM_E_INVALID, "dtype must be 32 or 64");
    if (d->n_bodies < 1) return fail(GSIM_E_INVALID, "n_bodies must be >= 1");
    if (d->n_particles < 1 || d->n_tets < 0 || d->n_tris < 0 || d->n_hinges < 0)
        return fail(GSIM_E_INVALID, "bad element counts");
    if (d->n_particles > INT32_MAX || 4 * (d->n_tets + d->n_hinges) + 3 * d->n_tris > INT32_MAX)
        return fail(GSIM_E_UNSUPPORTED, "model too large for 32-bit indices");
    if (!d->rest_x || !d->body_particle_off || !d->gravity || !d->dt) return fail(GSIM_E_INVALID, "NULL required array");
    if (d->n_tets && !d->tet_idx) return fail(GSIM_E_INVALID, "tet_idx is NULL");
    if (d->n_tris && !d->tri_idx) return fail(GSIM_E_INVALID, "tri_idx is NULL");
    if (d->n_hinges && !d->hinge_idx) return fail(GSIM_E_INVALID, "hinge_idx is NULL");
    const int nb = d->n_bodies;
    int rc;
    if ((rc = check_offsets(d->body_particle_off, nb, d->n_particles, "particle"))) return rc;
    if ((rc = check_offsets(d->body_tet_off, nb, d->n_tets, "tet"))) return rc;
    if ((rc = check_offsets(d->body_tri_off, nb, d->n_tris, "tri"))) return rc;
    if ((rc = check_offsets(d->body_hinge_off, nb, d->n_hinges, "hinge"))) return rc;
    if (d->tile_elems != 0 && (d->tile_elems < GSIM_TILE_MIN || d->tile_elems > GSIM_TILE_MAX))
        return fail(GSIM_E_INVALID, "tile_elems must be 0 or in [%d, %d]", GSIM_TILE_MIN, GSIM_TILE_MAX);
    P->tile_elems = d->tile_elems ? d->tile_elems : GSIM_TILE_DEFAULT;
    P->dtype = d->dtype;
    P->nb = nb;
    P->np = d->n_particles;
    P->ne = d->n_tets;
    P->nt = d->n_tris;
    P->nh = d->n_hinges;
    auto offs = [&](const int64_t* o) {
        std::vector<int64_t> v(nb + 1, 0);
        if (o) v.assign(o, o + nb + 1);
        return v;
    };
    P->poff = offs(d->body_particle_off);
    P->eoff = offs(d->body_tet_off);
    P->toff = offs(d->body_tri_off);
    P->hoff = offs(d->body_hinge_off);
    for (int b = 0; b < nb; ++b)
        if (P->poff[b + 1] == P->poff[b]) return fail(GSIM_E_INVALID, "body %d has no particles", b);

    std::vector<D3> X(P->np);
    for (int64_t i = 0; i < P->np; ++i) {
        X[i] = {d->rest_x[3 * i], d->rest_x[3 * i + 1], d->rest_x[3 * i + 2]};
        if (!finite(X[i].x) || !finite(X[i].y) || !finite(X[i].z))
            return fail(GSIM_E_NONFINITE, "rest position %lld is not finite", (long long)i);
    }
    P->rest.resize(3 * P->np);
    for (int64_t i = 0; i < P->np; ++i) {
        P->rest[3 * i] = X[i].x;
        P->rest[3 * i + 1] = X[i].y;
        P->rest[3 * i + 2] = X[i].z;
    }
    P->pinned.assign(P->np, 0);
    if (d->pinned)
        for (int64_t i = 0; i < P->np; ++i) P->pinned[i] = d->pinned[i] ? 1 : 0;
    P->dt.resize(nb);
    P->grav.resize(3 * nb);
    P->plane.resize(4 * nb);
    P->kb.resize(nb);
    P->contact_on.assign(nb, 0);
    P->air_on.assign(nb, 0);
    P->any_air = false;
    for (int b = 0; b < nb; ++b) {
        P->dt[b] = d->dt[b];
        if (!(d->dt[b] > 0) || !finite(d->dt[b])) return fail(GSIM_E_INVALID, "dt of body %d must be > 0", b);
        for (int c = 0; c < 3; ++c) {
            P->grav[3 * b + c] = d->gravity[3 * b + c];
            if (!finite(d->gravity[3 * b + c])) return fail(GSIM_E_NONFINITE, "gravity of body %d", b);
        }
        double pl[4] = {0.0, 1.0, 0.0, 0.0};
        if (d->ground)
            for (int c = 0; c < 4; ++c) pl[c] = d->ground[4 * b + c];
        double nn = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
        if (!(nn > 0) || !finite(nn) || !finite(pl[3])) return fail(GSIM_E_INVALID, "ground plane of body %d", b);
        for (int c = 0; c < 3; ++c) P->plane[4 * b + c] = pl[c] / nn;
        P->plane[4 * b + 3] = pl[3] / nn;
        P->kb[b] = d->k_bend ? d->k_bend[b] : 0.0;
        P->contact_on[b] = d->contact_on ? (d->contact_on[b] ? 1 : 0) : 0;
        P->air_on[b] = d->air_on ? (d->air_on[b] ? 1 : 0) : 0;
        P->any_air = P->any_air || P->air_on[b];
    }

    // element -> body checks
    auto in_body = [&](int64_t p, int b) { return p >= P->poff[b] && p < P->poff[b + 1]; };
    const int64_t ne = P->ne, nt = P->nt, nh = P->nh;
    P->tet_idx.resize(4 * ne);
    P->tet_dinv.resize(9 * ne);
    P->tet_vol.resize(ne);
    for (int b = 0; b < nb; ++b)
        for (int64_t e = P->eoff[b]; e < P->eoff[b + 1]; ++e) {
            int32_t id[4];
            for (int c = 0; c < 4; ++c) {
                id[c] = d->tet_idx[4 * e + c];
                if (!in_body(id[c], b)) return fail(GSIM_E_TOPOLOGY, "tet %lld corner %d outside body %d", (long long)e, c, b);
            }
            if (!distinct(id, 4)) return fail(GSIM_E_TOPOLOGY, "tet %lld repeats a particle", (long long)e);
            D3 c0 = sub(X[id[1]], X[id[0]]), c1 = sub(X[id[2]], X[id[0]]), c2 = sub(X[id[3]], X[id[0]]);
            double det = dt3(c0, crs(c1, c2));
            if (det < 0) {  // orient: swap corners 1 and 2
                std::swap(id[1], id[2]);
                std::swap(c0, c1);
                det = -det;
            }
            double h = std::max(std::max(nrm(c0), nrm(c1)), nrm(c2));
            if (!(det > 1e-12 * h * h * h)) return fail(GSIM_E_DEGENERATE, "tet %lld is degenerate", (long long)e);
            // Dm columns c0, c1, c2; inverse rows are (c1 x c2, c2 x c0, c0 x c1) / det
            D3 r[3] = {crs(c1, c2), crs(c2, c0), crs(c0, c1)};
            for (int i = 0; i < 3; ++i) {
                P->tet_dinv[(3 * i + 0) * ne + e] = r[i].x / det;
                P->tet_dinv[(3 * i + 1) * ne + e] = r[i].y / det;
                P->tet_dinv[(3 * i + 2) * ne + e] = r[i].z / det;
            }
            P->tet_vol[e] = det / 6.0;
            for (int c = 0; c < 4; ++c) P->tet_idx[c * ne + e] = id[c];
        }
    P->tri_idx.resize(3 * nt);
    P->tri_dinv.resize(4 * nt);
    P->tri_area.resize(nt);
    for (int b = 0; b < nb; ++b)
        for (int64_t t = P->toff[b]; t < P->toff[b + 1]; ++t) {
            int32_t id[3];
            for (int c = 0; c < 3; ++c) {
                id[c] = d->tri_idx[3 * t + c];
                if (!in_body(id[c], b)) return fail(GSIM_E_TOPOLOGY, "tri %lld corner %d outside body %d", (long long)t, c, b);
            }
            if (!distinct(id, 3)) return fail(GSIM_E_TOPOLOGY, "tri %lld repeats a particle", (long long)t);
            D3 a = sub(X[id[1]], X[id[0]]), c = sub(X[id[2]], X[id[0]]);
            D3 n = crs(a, c);
            double la = nrm(a), ln = nrm(n);
            if (!(la > 0) || !(ln > 1e-12 * la * nrm(c))) return fail(GSIM_E_DEGENERATE, "tri %lld is degenerate", (long long)t);
            D3 e1 = {a.x / la, a.y / la, a.z / la};
            D3 nn = {n.x / ln, n.y / ln, n.z / ln};
            D3 e2 = crs(nn, e1);
            // Dm = [[e1.a, e1.c], [e2.a, e2.c]]; e2.a = 0 by construction
            double m00 = dt3(e1, a), m01 = dt3(e1, c), m10 = dt3(e2, a), m11 = dt3(e2, c);
            double det = m00 * m11 - m01 * m10;
            P->tri_dinv[0 * nt + t] = m11 / det;
            P->tri_dinv[1 * nt + t] = -m01 / det;
            P->tri_dinv[2 * nt + t] = -m10 / det;
            P->tri_dinv[3 * nt + t] = m00 / det;
            P->tri_area[t] = 0.5 * det;
            for (int k = 0; k < 3; ++k) P->tri_idx[k * nt + t] = id[k];
        }
    P->hin_idx.resize(4 * nh);
    P->hin_phi0.resize(nh);
    for (int b = 0; b < nb; ++b)
        for (int64_t h = P->hoff[b]; h < P->hoff[b + 1]; ++h) {
            int32_t id[4];
            D3 x[4];
            for (int c = 0; c < 4; ++c) {
                id[c] = d->hinge_idx[4 * h + c];
                if (!in_body(id[c], b))
                    return fail(GSIM_E_TOPOLOGY, "hinge %lld corner %d outside body %d", (long long)h, c, b);
                x[c] = X[id[c]];
            }
            if (!distinct(id, 4)) return fail(GSIM_E_TOPOLOGY, "hinge %lld repeats a particle", (long long)h);
            D3 E = sub(x[3], x[2]);
            double el = nrm(E);
            double n1 = nrm(crs(sub(x[0], x[2]), sub(x[0], x[3]))), n2 = nrm(crs(sub(x[1], x[3]), sub(x[1], x[2])));
            if (!(el > 0) || !(n1 > 1e-12 * el * el) || !(n2 > 1e-12 * el * el))
                return fail(GSIM_E_DEGENERATE, "hinge %lld is degenerate", (long long)h);
            P->hin_phi0[h] = rest_angle(x);
            for (int c = 0; c < 4; ++c) P->hin_idx[c * nh + h] = id[c];
        }

    if (int rc = build_tiles(P)) return rc;
    if (fused) {
        colour_elements(P);
    } else {
        P->fused_ok = P->coloured = false;
        P->cbase.assign(3 * nb, 0);
        P->ncol.assign(3 * nb, 0);
    }
    return GSIM_OK;
}

// ---------------------------------------------------------------- layout ---
const int MIN_TILE = 64;  // smallest tile (block 64, 1 item): bounds the tile-list capacity

// (each launch lane pads its list to a multiple of N_XCD)
int64_t tile_capacity(const gsim_plan* P, bool particles) {
    if (!particles) return (int64_t)P->etiles.size() + 2 * MAX_LANES * N_XCD;  // element tiles are planned
    int64_t n = 0;
    for (int b = 0; b < P->nb; ++b) n += (P->poff[b + 1] - P->poff[b] + MIN_TILE - 1) / MIN_TILE;
    return n + 2 * MAX_LANES * N_XCD;
}


template <typename T>
Layout make_layout(const gsim_plan* P, int max_steps) {
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        o = align_up(o, 256);
        size_t at = o;
        o += bytes;
        return at;
    };
    const int64_t ne = P->ne, nt = P->nt, nh = P->nh, np = P->np;
    const int64_t cap_p = tile_capacity(P, true), cap_e = tile_capacity(P, false);
    L.model = take(sizeof(ModelDev<T>));
    L.bodies = take(sizeof(BodyDev<T>) * P->nb);
    L.etiles = take(sizeof(Tile) * cap_e);
    L.ptiles = take(sizeof(Tile) * cap_p);
    L.tet_code = take(4 * ne * 4);
    L.tet_dinv = take(9 * ne * sizeof(T));
    L.tet_vol = take(ne * sizeof(T));
    L.tri_code = take(3 * nt * 4);
    L.tri_dinv = take(4 * nt * sizeof(T));
    L.tri_area = take(nt * sizeof(T));
    L.hin_code = take(4 * nh * 4);
    L.hin_phi0 = take(nh * sizeof(T));
    L.tp = take(P->tp_id.size() * 12 + 16);
    L.gbase = take(P->gbase.size() * 4 + 4);
    L.pdeg = take(np * 4);
    L.pinned = take(np);
    L.rest = take(3 * np * sizeof(T));
    L.rgap = take(np * sizeof(T));
    L.bflag = take(2 * (size_t)P->nb * 4);
    L.slots = take(4 * std::max<int64_t>(P->nslot, 1) * sizeof(T));
    L.fslots = take(3 * std::max<int64_t>(P->nslot, 1) * sizeof(T));
    L.vslots = P->any_air ? take(4 * std::max<int64_t>(P->nslot, 1) * sizeof(T)) : 0;
    L.cpart = take(4 * (cap_p + 1) * sizeof(T));
    L.lpart = take((cap_p + 1) * sizeof(T));
    L.fbuf = take(2 * 6 * np * sizeof(T));
    L.abuf = take(2 * 6 * np * sizeof(T));
    L.fbar = take(2 * 3 * np * sizeof(T));
    L.f_tet_idx = take(4 * ne * 4);
    L.f_tet_dinv = take(9 * ne * sizeof(T));
    L.f_tet_vol = take(ne * sizeof(T));
    L.f_tet_orig = take(ne * 4);
    L.f_tri_idx = take(3 * nt * 4);
    L.f_tri_dinv = take(4 * nt * sizeof(T));
    L.f_tri_area = take(nt * sizeof(T));
    L.f_tri_orig = take(nt * 4);
    L.f_hin_idx = take(4 * nh * 4);
    L.f_hin_phi0 = take(nh * sizeof(T));
    L.f_hin_orig = take(nh * 4);
    L.coff = take(P->coff.size() * 4 + 4);
    L.border = take(P->nb * 4 + 4);
    L.f_par = take(3 * ne * sizeof(T));
    L.f_ktri = take(nt * sizeof(T));
    L.f_g = take(3 * ne * sizeof(T));
    L.f_gk = take(nt * sizeof(T));
    L.f_hpar = take(nh * sizeof(T));
    L.f_gh = take(nh * sizeof(T));
    L.ntiles = take(sizeof(Tile) * (cap_e + cap_p));  // natural-order tiles (persistent execution)
    L.toff = take(2 * (P->nb + 1) * 4);
    L.table_cap = 4 * (int64_t)max_steps + 8;
    L.table = take(sizeof(StepDev<T>) * L.table_cap);
    L.total = align_up(o, 256);
    return L;
}

}  // namespace


namespace {

// Natural-order tile list of one pass.  Element tiles are the plan's; particle
// tiles are `tile`-sized chunks of each body's particles and get consecutive
// partial-buffer rows.
void natural_tiles(const gsim_model* m, bool particles, int tile, std::vector<Tile>& nat, int& rows) {
    nat.clear();
    rows = 0;
    if (!particles) {
        nat = m->etiles_plan;
        return;
    }
    for (int b = 0; b < m->nb; ++b)
        for (int64_t s = m->poff[b]; s < m->poff[b + 1]; s += tile) {
            Tile t{};
            t.model = 0;
            t.body = b;
            t.kind = TILE_PART;
            t.count = (int32_t)std::min<int64_t>(tile, m->poff[b + 1] - s);
            t.begin = s;
            t.id = rows++;
            nat.push_back(t);
        }
}

template <typename T>
int upload_tiles(gsim_model* m, void* stream, UploadSink* sink = nullptr) {
    std::vector<Tile> et, pt;
    int rows_e = 0;
    natural_tiles(m, false, 0, m->etiles_nat, rows_e);
    natural_tiles(m, true, m->pblock * m->pitems, m->ptiles_nat, m->n_ptile_rows);
    // launch lanes: bodies assigned largest first to the lane with the least work so
    // far; each lane's tiles are XCD-ordered on their own and the lists concatenated
    std::vector<int> lane(m->nb, 0);
    if (m->lanes > 1) {
        std::vector<int> order(m->nb);
        for (int b = 0; b < m->nb; ++b) order[b] = b;
        auto work = [&](int b) {
            return (m->eoff[b + 1] - m->eoff[b]) + (m->toff[b + 1] - m->toff[b]) + (m->hoff[b + 1] - m->hoff[b]) +
                   (m->poff[b + 1] - m->poff[b]);
        };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
        int64_t load[MAX_LANES] = {};
        for (int b : order) {
            int l = 0;
            for (int k = 1; k < m->lanes; ++k)
                if (load[k] < load[l]) l = k;
            lane[b] = l;
            load[l] += work(b);
        }
    }
    // per lane: the plain bodies' tiles, then the air bodies' (each group XCD-ordered)
    auto by_lane = [&](const std::vector<Tile>& nat, int kind, int dummy, std::vector<Tile>& out, int* bounds,
                       int* air_from) {
        out.clear();
        for (int l = 0; l <= MAX_LANES; ++l) bounds[l] = 0;
        for (int l = 0; l < MAX_LANES; ++l) air_from[l] = 0;
        for (int l = 0; l < m->lanes; ++l) {
            for (int air = 0; air < 2; ++air) {
                std::vector<Tile> mine, ord;
                for (const Tile& t : nat)
                    if (lane[t.body] == l && (m->air_on[t.body] != 0) == (air != 0)) mine.push_back(t);
                if (air) air_from[l] = (int)out.size();
                if (mine.empty()) continue;
                int grid = 0;
                xcd_order(mine, kind, dummy, ord, grid);
                out.insert(out.end(), ord.begin(), ord.begin() + grid);
            }
            bounds[l + 1] = (int)out.size();
        }
    };
    by_lane(m->etiles_nat, TILE_TET, 0, et, m->lane_e, m->lane_e_air);
    by_lane(m->ptiles_nat, TILE_PART, m->n_ptile_rows, pt, m->lane_p, m->lane_p_air);
    m->n_etiles = m->lane_e[m->lanes];
    m->n_ptiles = m->lane_p[m->lanes];
    hipStream_t s = (hipStream_t)stream;
    auto up = [&](void* dst, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return sink ? sink->copy(dst, src, n) : hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
    };
    HIP_TRY(up(m->ws + m->L.etiles, et.data(), et.size() * sizeof(Tile)), "upload tiles");
    HIP_TRY(up(m->ws + m->L.ptiles, pt.data(), pt.size() * sizeof(Tile)), "upload tiles");
    // persistent execution: the natural-order tiles (element, then particle) and each
    // body's ranges in them
    {
        std::vector<Tile> nat(m->etiles_nat);
        nat.insert(nat.end(), m->ptiles_nat.begin(), m->ptiles_nat.end());
        std::vector<int32_t> toff(2 * (m->nb + 1), 0);
        for (const Tile& t : m->etiles_nat) toff[t.body + 1]++;
        for (const Tile& t : m->ptiles_nat) toff[m->nb + 1 + t.body + 1]++;
        for (int b = 0; b < m->nb; ++b) {
            toff[b + 1] += toff[b];
            toff[m->nb + 1 + b + 1] += toff[m->nb + 1 + b];
        }
        m->n_etiles_nat = (int)m->etiles_nat.size();
        HIP_TRY(up(m->ws + m->L.ntiles, nat.data(), nat.size() * sizeof(Tile)), "upload tiles");
        HIP_TRY(up(m->ws + m->L.toff, toff.data(), toff.size() * 4), "upload tiles");
    }
    // body particle-tile ranges (contact / loss partial rows) depend on the tile size
    BodyDev<T>* bodies = reinterpret_cast<BodyDev<T>*>(m->bodies_host.data());
    int row = 0;
    const int tile = m->pblock * m->pitems;
    for (int b = 0; b < m->nb; ++b) {
        bodies[b].pt0 = row;
        row += (int)((m->poff[b + 1] - m->poff[b] + tile - 1) / tile);
        bodies[b].pt1 = row;
    }
    HIP_TRY(up(m->ws + m->L.bodies, bodies, sizeof(BodyDev<T>) * m->nb), "upload bodies");
    if (!sink) HIP_TRY(hipStreamSynchronize(s), "sync");
    for (auto& g : m->graphs)
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
    m->graphs.clear();
    return GSIM_OK;
}


// ------------------------------------------------------------- launching ---
template <typename T>
struct Ctx {
    gsim_model* m;
    const ModelDev<T>* md;
    const StepDev<T>* table;
    const Tile* et;
    const Tile* pt;
    T* fbuf;  // [2][6][np]
    T* abuf;
    int64_t np;
};

template <typename T>
Ctx<T> ctx(gsim_model* m) {
    Ctx<T> c;
    c.m = m;
    c.md = (const ModelDev<T>*)(m->ws + m->L.model);
    c.table = (const StepDev<T>*)(m->ws + m->L.table);
    c.et = (const Tile*)(m->ws + m->L.etiles);
    c.pt = (const Tile*)(m->ws + m->L.ptiles);
    c.fbuf = (T*)(m->ws + m->L.fbuf);
    c.abuf = (T*)(m->ws + m->L.abuf);
    c.np = m->np;
    return c;
}

// Shared adjoint + recompute element launches pair each tile's two passes in one
// workgroup when the model has at least this many element tiles (8 per CU): measured,
// the paired layout is faster for the 256- and 2048-body batches (2,794 and ~21,000
// tiles) and slower for the 200k-tet blob (800 tiles), the tiny cube and the cloth.
const int DUAL_PAIR_MIN_TILES = 2048;

// One launch of the sequence a call replays: pass kind and its table row.
enum Op : int {
    OP_FWD = 0,
    OP_ADJ = 1,
    OP_FILL_CPART = 2,
    OP_CONTACT_REDUCE = 3,
    OP_LOSS = 4,
    OP_FUSED_FWD = 5,  // whole segment of forward steps, one workgroup per body
    OP_FUSED_ADJ = 6,    // whole segment of adjoint steps, one workgroup per body
    OP_FUSED_PARAMS = 7, // parameters into colour order (and colour-ordered gradient clear)
    OP_FUSED_GRADS = 8,  // colour-ordered gradients back to element order
    OP_FUSED_ADJ_ACT = 9, // OP_FUSED_ADJ that also accumulates actuation gradients
    OP_DUAL = 10          // adjoint pass of `row` and forward pass of `row2` in the same launches
};

template <typename T>
size_t fused_lds(const gsim_model* m, bool adjoint) {
    return m->fused_dyn[adjoint ? 1 : 0];
}
struct Launch {
    int op;
    int64_t row;
    int64_t row2 = 0;  // OP_DUAL: the forward pass's row
};

hipError_t take_event(gsim_model* m, hipEvent_t* e) {
    if (!m->evt_pool.empty()) {
        *e = m->evt_pool.back();
        m->evt_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Launches one pass, bracketed by timing events when kernel `k` is selected.
template <typename F>
int timed(gsim_model* m, int k, void* stream, F launch) {
    if (!(m->timing_mask & (1 << k))) return launch();
    hipEvent_t a, b;
    HIP_TRY(take_event(m, &a), "timing event");
    HIP_TRY(take_event(m, &b), "timing event");
    // the kernel itself records a and b as its start and end; a pass with nothing to
    // launch records them back to back
    arm_launch_events(a, b);
    int rc = launch();
    if (!disarm_launch_events()) {
        HIP_TRY(hipEventRecord(a, (hipStream_t)stream), "timing record");
        HIP_TRY(hipEventRecord(b, (hipStream_t)stream), "timing record");
    }
    m->pending.push_back({k, a, b});
    return rc;
}

// Launch sequences.  Forward and adjoint passes of consecutive steps run on the
// model's lanes when it has more than one: lane 0 on the caller's stream, lane l
// on the model's lane stream l, forked from the caller's stream before the first
// such pass and joined back before any launch that spans all bodies (and at the
// end).  The lanes hold disjoint bodies, so results do not depend on the lanes.
// With kernel timing on, each pass is one launch over all lanes' tiles.
template <typename T>
int run_sequence(gsim_model* m, const std::vector<Launch>& seq, void* stream) {
    Ctx<T> c = ctx<T>(m);
    const ModelDev<T>* md = c.md;
    const int nl = m->timing_mask == 0 ? m->lanes : 1;
    hipStream_t s0 = (hipStream_t)stream;
    bool forked = false;
    auto join = [&]() -> int {
        if (forked) {
            for (int l = 1; l < nl; ++l) {
                HIP_TRY(hipEventRecord(m->ev_join[l], m->lane_stream[l]), "join lanes");
                HIP_TRY(hipStreamWaitEvent(s0, m->ev_join[l], 0), "join lanes");
            }
            forked = false;
        }
        return GSIM_OK;
    };
    // one pass over lane l's tiles (l < 0: all tiles, one launch)
    // One pass over the tile ranges [e0, e1) / [p0, p1) on stream st: element passes
    // and the particle adjoint launch the plain tiles [x0, xa) and the air bodies'
    // tiles [xa, x1) with their kernel variants (one launch when either is empty).
    auto ranges = [&](int e0, int ea, int e1, int p0, int pa, int p1, void* st, const StepDev<T>* sd,
                      bool adjoint) -> int {
        const size_t wf = m->etile_words[0] * sizeof(T), wa = m->etile_words[1] * sizeof(T);
        if (!adjoint) {
            if (ea > e0) LAUNCH_TRY(timed(m, 0, st, [&] { return launch_elem_fwd<T>(md, sd, c.et + e0, ea - e0, m->block, wf, false, st); }), "element pass");
            if (e1 > ea) LAUNCH_TRY(timed(m, 0, st, [&] { return launch_elem_fwd<T>(md, sd, c.et + ea, e1 - ea, m->block, wf, true, st); }), "element pass");
            LAUNCH_TRY(timed(m, 1, st, [&] { return launch_part_fwd<T>(md, sd, c.pt + p0, p1 - p0, m->pblock, m->pitems, st); }), "particle pass");
        } else {
            if (ea > e0) LAUNCH_TRY(timed(m, 2, st, [&] { return launch_elem_adj<T>(md, sd, c.et + e0, ea - e0, m->block, wa, false, st); }), "element adjoint");
            if (e1 > ea) LAUNCH_TRY(timed(m, 2, st, [&] { return launch_elem_adj<T>(md, sd, c.et + ea, e1 - ea, m->block, wa, true, st); }), "element adjoint");
            if (pa > p0) LAUNCH_TRY(timed(m, 3, st, [&] { return launch_part_adj<T>(md, sd, c.pt + p0, pa - p0, m->pblock, m->pitems, false, st); }), "particle adjoint");
            if (p1 > pa) LAUNCH_TRY(timed(m, 3, st, [&] { return launch_part_adj<T>(md, sd, c.pt + pa, p1 - pa, m->pblock, m->pitems, true, st); }), "particle adjoint");
        }
        return GSIM_OK;
    };
    // one pass of lane l on its stream; l < 0: every lane on the caller's stream, as
    // one launch per kernel when no body has air
    auto pass = [&](int l, const StepDev<T>* sd, bool adjoint) -> int {
        if (l >= 0)
            return ranges(m->lane_e[l], m->lane_e_air[l], m->lane_e[l + 1], m->lane_p[l], m->lane_p_air[l],
                          m->lane_p[l + 1], l > 0 ? (void*)m->lane_stream[l] : stream, sd, adjoint);
        if (!m->any_air) return ranges(0, m->n_etiles, m->n_etiles, 0, m->n_ptiles, m->n_ptiles, stream, sd, adjoint);
        for (int k = 0; k < m->lanes; ++k)
            if (int rc = ranges(m->lane_e[k], m->lane_e_air[k], m->lane_e[k + 1], m->lane_p[k], m->lane_p_air[k],
                                m->lane_p[k + 1], stream, sd, adjoint))
                return rc;
        return GSIM_OK;
    };
    // adjoint pass of row sd_a and forward pass of row sd_f, element launch then particle
    // launch, over lane l's tiles (l < 0: every tile, one pair of launches); models
    // without lift/drag only
    auto dual = [&](int l, const StepDev<T>* sd_a, const StepDev<T>* sd_f) -> int {
        const int e0 = l < 0 ? 0 : m->lane_e[l], e1 = l < 0 ? m->n_etiles : m->lane_e[l + 1];
        const int p0 = l < 0 ? 0 : m->lane_p[l], p1 = l < 0 ? m->n_ptiles : m->lane_p[l + 1];
        void* st = l > 0 ? (void*)m->lane_stream[l] : stream;
        const size_t lds = std::max(m->etile_words[0], m->etile_words[1]) * sizeof(T);
        // a model with many element tiles pairs each tile's two passes in one workgroup
        // (its records read once); with few, both passes of a tile run side by side
        const bool paired = m->n_etiles >= DUAL_PAIR_MIN_TILES;
        LAUNCH_TRY(timed(m, 6, st, [&] {
            return launch_dual<T>(md, sd_a, sd_f, c.et + e0, e1 - e0, c.pt + p0, p1 - p0, m->block, m->pblock, lds,
                                  false, paired, st);
        }), "overlapped element passes");
        LAUNCH_TRY(timed(m, 7, st, [&] {
            return launch_dual<T>(md, sd_a, sd_f, c.et + e0, e1 - e0, c.pt + p0, p1 - p0, m->block, m->pblock, lds,
                                  true, false, st);
        }), "overlapped particle passes");
        return GSIM_OK;
    };
    for (size_t li = 0; li < seq.size(); ++li) {
        const Launch& l = seq[li];
        const StepDev<T>* sd = c.table + l.row;
        if (l.op == OP_DUAL) {
            if (nl == 1) {
                if (int rc = dual(-1, sd, c.table + l.row2)) return rc;
                continue;
            }
            if (!forked) {
                HIP_TRY(hipEventRecord(m->ev_fork, s0), "fork lanes");
                for (int k = 1; k < nl; ++k) HIP_TRY(hipStreamWaitEvent(m->lane_stream[k], m->ev_fork, 0), "fork lanes");
                forked = true;
            }
            for (int k = 0; k < nl; ++k)
                if (int rc = dual(k, sd, c.table + l.row2)) return rc;
            continue;
        }
        if (m->exec == GSIM_EXEC_PERSIST && (l.op == OP_FWD || l.op == OP_ADJ)) {
            // the run of forward / adjoint steps on consecutive rows: one launch
            size_t lj = li + 1;
            while (lj < seq.size() && (seq[lj].op == OP_FWD || seq[lj].op == OP_ADJ) &&
                   seq[lj].row == seq[lj - 1].row + 1)
                ++lj;
            const Tile* nt = reinterpret_cast<const Tile*>(m->ws + m->L.ntiles);
            const size_t lds = std::max(m->etile_words[0], m->etile_words[1]) * sizeof(T);
            // the particle passes' block size, so each thread sums the same particles into
            // the contact-gradient reduction as in the two-pass launches (element results do
            // not depend on the block size)
            LAUNCH_TRY(launch_persist<T>(md, sd, (int)(lj - li), nt, nt + m->n_etiles_nat,
                                         reinterpret_cast<const int32_t*>(m->ws + m->L.toff), m->nb, m->pblock, lds,
                                         stream),
                       "persistent steps");
            li = lj - 1;
            continue;
        }
        if (l.op == OP_FWD || l.op == OP_ADJ) {
            const bool adjoint = l.op == OP_ADJ;
            if (nl == 1) {
                if (int rc = pass(-1, sd, adjoint)) return rc;
                continue;
            }
            if (!forked) {
                HIP_TRY(hipEventRecord(m->ev_fork, s0), "fork lanes");
                for (int k = 1; k < nl; ++k) HIP_TRY(hipStreamWaitEvent(m->lane_stream[k], m->ev_fork, 0), "fork lanes");
                forked = true;
            }
            for (int k = 0; k < nl; ++k)
                if (int rc = pass(k, sd, adjoint)) return rc;
            continue;
        }
        if (int rc = join()) return rc;
        switch (l.op) {
            case OP_FILL_CPART:
                LAUNCH_TRY(launch_fill<T>((T*)(m->ws + m->L.cpart), 4 * (int64_t)(m->n_ptile_rows + 1), T(0), stream), "clear");
                break;
            case OP_CONTACT_REDUCE:
                LAUNCH_TRY(launch_contact_reduce<T>(md, sd, m->nb, stream), "contact reduce");
                break;
            case OP_FUSED_FWD:
                LAUNCH_TRY(timed(m, 4, stream, [&] {
                    return launch_fused_fwd<T>(md, sd, (const int32_t*)(m->ws + m->L.border), m->nb, fused_lds<T>(m, false), stream);
                }), "fused forward");
                break;
            case OP_FUSED_ADJ:
            case OP_FUSED_ADJ_ACT:
                LAUNCH_TRY(timed(m, 5, stream, [&] {
                    return launch_fused_adj<T>(md, sd, (const int32_t*)(m->ws + m->L.border), m->nb,
                                               fused_lds<T>(m, true), l.op == OP_FUSED_ADJ_ACT, stream);
                }), "fused adjoint");
                break;
            case OP_FUSED_PARAMS:
                LAUNCH_TRY(launch_fused_params<T>(md, sd, stream), "fused parameters");
                break;
            case OP_FUSED_GRADS:
                LAUNCH_TRY(launch_fused_grads<T>(md, sd, stream), "fused gradients");
                break;
            case OP_LOSS:
                LAUNCH_TRY(launch_loss<T>(md, sd, c.pt, m->n_ptiles, m->pblock, m->pitems, m->nb, stream), "loss");
                break;
        }
    }
    return join();
}

// Uploads table rows [row0, row0 + n) if they differ from the last upload.  The
// pinned stage doubles as the record of what the device holds; before it is
// rewritten the previous upload must have finished reading it.
template <typename T>
int upload_rows(gsim_model* m, int64_t row0, const std::vector<StepDev<T>>& rows, void* stream) {
    const size_t off = (size_t)row0 * sizeof(StepDev<T>), n = rows.size() * sizeof(StepDev<T>);
    if (row0 + (int64_t)rows.size() > m->L.table_cap) return fail(GSIM_E_WORKSPACE, "launch table too small");
    if (!m->stage) {  // the pinned stage is made on the first upload (models driven by the
                      // serving engine, which keeps its own tables, never need one)
        const size_t cap = sizeof(StepDev<T>) * m->L.table_cap;
        HIP_TRY(hipHostMalloc((void**)&m->stage, cap, hipHostMallocDefault), "launch table stage");
        std::memset(m->stage, 0, cap);
        if (n == 0) return GSIM_OK;
    } else if (n == 0 || std::memcmp(m->stage + off, rows.data(), n) == 0) {
        return GSIM_OK;
    }
    HIP_TRY(hipEventSynchronize(m->stage_evt), "wait for table upload");
    std::memcpy(m->stage + off, rows.data(), n);
    HIP_TRY(hipMemcpyAsync(m->ws + m->L.table + off, m->stage + off, n, hipMemcpyHostToDevice, (hipStream_t)stream),
            "upload launch table");
    HIP_TRY(hipEventRecord(m->stage_evt, (hipStream_t)stream), "record table upload");
    return GSIM_OK;
}

// Runs a launch sequence, through a cached hipGraph when the model asks for it.
template <typename T>
int execute(gsim_model* m, long long key, const std::vector<Launch>& seq, void* stream) {
    if (m->exec == GSIM_EXEC_GRAPH) {
        if (m->timing_mask) return fail(GSIM_E_UNSUPPORTED, "kernel timing needs plain execution");
        if (stream == nullptr) return fail(GSIM_E_UNSUPPORTED, "graph execution needs a non-default stream");
        auto it = m->graphs.find(key);
        if (it == m->graphs.end()) {
            hipStream_t s = (hipStream_t)stream;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
            int rc = run_sequence<T>(m, seq, stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "end capture");
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e, "instantiate graph");
            it = m->graphs.emplace(key, GraphEntry{ex}).first;
        }
        HIP_TRY(hipGraphLaunch(it->second.exec, (hipStream_t)stream), "graph launch");
        return GSIM_OK;
    }
    return run_sequence<T>(m, seq, stream);
}

template <typename T>
void fill_params(StepDev<T>& r, const gsim_params* p, const gsim_grads* g) {
    r.mu = (const T*)p->mu;
    r.lam = (const T*)p->lam;
    r.act = (const T*)p->act;
    r.ktri = (const T*)p->k_tri;
    r.mass = (const T*)p->mass;
    r.contact = (const T*)p->contact;
    r.hact = (const T*)p->hact;
    r.air = (const T*)p->air;
    if (g) {
        r.g_mu = (T*)g->mu;
        r.g_lam = (T*)g->lam;
        r.g_ktri = (T*)g->k_tri;
        r.g_mass = (T*)g->mass;
        r.g_contact = (T*)g->contact;
        r.g_act = (T*)g->act;
        r.g_hact = (T*)g->hact;
    }
}

// Step t of a call reads (and accumulates into) the actuation arrays of step t.
template <typename T>
void at_step(StepDev<T>& r, const gsim_params* p, const gsim_grads* g, int64_t t) {
    if (p->act) r.act = (const T*)p->act + t * p->act_stride;
    if (p->hact) r.hact = (const T*)p->hact + t * p->hact_stride;
    if (g && g->act) r.g_act = (T*)g->act + t * g->act_stride;
    if (g && g->hact) r.g_hact = (T*)g->hact + t * g->hact_stride;
}

int check_params(const gsim_model* m, const gsim_params* p, const gsim_grads* g = nullptr) {
    if (!p) return fail(GSIM_E_INVALID, "NULL params");
    if (p->act_stride < 0 || p->hact_stride < 0 || (g && (g->act_stride < 0 || g->hact_stride < 0)))
        return fail(GSIM_E_INVALID, "actuation strides must be >= 0");
    const bool per_step = (p->act && p->act_stride) || (p->hact && p->hact_stride) ||
                          (g && ((g->act && g->act_stride) || (g->hact && g->hact_stride)));
    if (m->exec == GSIM_EXEC_FUSED && per_step)
        return fail(GSIM_E_UNSUPPORTED, "the fused path takes one actuation array for all steps (strides must be 0)");
    if (g && ((g->mu && (g->mu == g->lam || g->mu == g->act)) || (g->lam && g->lam == g->act)))
        return fail(GSIM_E_INVALID, "the mu, lam and act gradient buffers must be distinct");
    if (m->ne && (!p->mu || !p->lam)) return fail(GSIM_E_INVALID, "mu and lam are required for tets");
    if (m->nt && !p->k_tri) return fail(GSIM_E_INVALID, "k_tri is required for triangles");
    if (!p->mass) return fail(GSIM_E_INVALID, "mass is required");
    if (!p->contact) return fail(GSIM_E_INVALID, "contact parameters are required ([n_bodies][4])");
    if (m->any_air && !p->air) return fail(GSIM_E_INVALID, "air coefficients are required ([n_bodies][2]): a body has air_on");
    return GSIM_OK;
}

// The second segment buffer is in use (kept last segment; overlapped recompute under
// plain and graph execution): models without lift/drag, two-pass or persistent execution.
bool uses_seg2(const gsim_model* m) {
    return m->seg2 && !m->any_air &&
           (m->exec == GSIM_EXEC_PLAIN || m->exec == GSIM_EXEC_GRAPH || m->exec == GSIM_EXEC_PERSIST);
}

// table regions
int64_t region_rollout(const gsim_model*) { return 0; }
int64_t region_backward(const gsim_model* m) { return m->max_steps + 2; }
int64_t region_step(const gsim_model* m) { return 3 * (int64_t)m->max_steps + 4; }
int64_t region_misc(const gsim_model* m) { return 4 * (int64_t)m->max_steps + 6; }

// Fused-path sequences: each launch runs a whole segment of steps for every body.
template <typename T>
StepDev<T> fused_row(const gsim_params* p, const gsim_grads* g) {
    StepDev<T> r;
    std::memset(&r, 0, sizeof r);
    fill_params<T>(r, p, g);
    return r;
}

template <typename T>
int do_fused_forward(gsim_model* m, const gsim_params* p, const T* x, const T* v, T* xo, T* vo, T* ckpt, int n,
                     int64_t row0, long long key, void* stream) {
    std::vector<StepDev<T>> rows(1, fused_row<T>(p, nullptr));
    StepDev<T>& r = rows[0];
    r.x = x;
    r.v = v;
    r.x_abs = 1;
    r.xo = xo;
    r.vo = vo;
    r.xo_abs = 1;
    r.ckx = ckpt;
    r.ckv = ckpt ? ckpt + 3 * m->np : nullptr;
    r.ckpt_every = m->K;
    r.nsteps = n;
    r.t_base = 0;
    int rc = upload_rows<T>(m, row0, rows, stream);
    if (rc) return rc;
    std::vector<Launch> seq{{OP_FUSED_PARAMS, row0}, {OP_FUSED_FWD, row0}};
    return execute<T>(m, key, seq, stream);
}

template <typename T>
int do_fused_rollout_backward(gsim_model* m, const gsim_params* p, const T* ck, int n, T* seg, gsim_state af,
                              gsim_state ai, const gsim_grads* g, void* stream) {
    Ctx<T> c = ctx<T>(m);
    const int64_t S = 6 * c.np, np = c.np;
    const int K = m->K, nseg = (n + K - 1) / K;
    const bool act = g && (g->act || g->hact);
    std::vector<StepDev<T>> rows(1, fused_row<T>(p, g));
    const int64_t r0 = region_backward(m);
    std::vector<Launch> seq{{OP_FUSED_PARAMS, r0}};
    for (int s = nseg - 1, q = 0; s >= 0; --s, ++q) {
        const int t0 = s * K, L = std::min(n, t0 + K) - t0;
        if (L > 1) {  // recompute states t0+1 .. t0+L-1 into seg[0 .. L-2]
            StepDev<T> r = fused_row<T>(p, nullptr);
            r.x = ck + s * S;
            r.v = r.x + 3 * np;
            r.seg = seg;
            r.nsteps = L - 1;
            r.t_base = t0;
            r.ckpt_every = K;
            rows.push_back(r);
            seq.push_back({OP_FUSED_FWD, r0 + (int64_t)rows.size() - 1});
        }
        StepDev<T> r = fused_row<T>(p, g);
        r.x = ck + s * S;
        r.v = r.x + 3 * np;
        r.seg_in = seg;
        r.nsteps = L;
        r.t_base = t0;
        r.ckpt_every = K;
        if (q == 0) {
            r.xb = (const T*)af.x;
            r.vb = (const T*)af.v;
        } else {
            r.xb = c.abuf + ((q - 1) & 1) * S;
            r.vb = r.xb + 3 * np;
        }
        if (s == 0) {
            r.xbo = (T*)ai.x;
            r.vbo = (T*)ai.v;
        } else {
            r.xbo = c.abuf + (q & 1) * S;
            r.vbo = r.xbo + 3 * np;
        }
        rows.push_back(r);
        seq.push_back({act ? OP_FUSED_ADJ_ACT : OP_FUSED_ADJ, r0 + (int64_t)rows.size() - 1});
    }
    seq.push_back({OP_FUSED_GRADS, r0});
    int rc = upload_rows<T>(m, r0, rows, stream);
    if (rc) return rc;
    return execute<T>(m, (7LL << 40) | ((long long)n << 1) | (act ? 1 : 0), seq, stream);
}

template <typename T>
int do_step(gsim_model* m, const gsim_params* p, gsim_state in, gsim_state out, int n, void* stream) {
    if (n < 1 || n > m->max_steps) return fail(GSIM_E_INVALID, "n_steps must be in [1, %d]", m->max_steps);
    if (!in.x || !in.v || !out.x || !out.v) return fail(GSIM_E_INVALID, "NULL state");
    int rc = check_params(m, p);
    if (rc) return rc;
    if (m->exec == GSIM_EXEC_FUSED)
        return do_fused_forward<T>(m, p, (const T*)in.x, (const T*)in.v, (T*)out.x, (T*)out.v, nullptr, n, region_step(m),
                                   (8LL << 40) | n, stream);
    Ctx<T> c = ctx<T>(m);
    const int64_t S = 6 * c.np;
    std::vector<StepDev<T>> rows(n);
    std::vector<Launch> seq;
    const int64_t r0 = region_step(m);
    for (int t = 0; t < n; ++t) {
        StepDev<T>& r = rows[t];
        std::memset(&r, 0, sizeof r);
        fill_params<T>(r, p, nullptr);
        at_step<T>(r, p, nullptr, t);
        if (t == 0) {
            r.x = (const T*)in.x;
            r.v = (const T*)in.v;
            r.x_abs = 1;
        } else {
            r.x = c.fbuf + ((t - 1) & 1) * S;
            r.v = r.x + 3 * c.np;
        }
        if (t == n - 1) {
            r.xo = (T*)out.x;
            r.vo = (T*)out.v;
            r.xo_abs = 1;
        } else {
            r.xo = c.fbuf + (t & 1) * S;
            r.vo = r.xo + 3 * c.np;
        }
        seq.push_back({OP_FWD, r0 + t});
    }
    if ((rc = upload_rows<T>(m, r0, rows, stream))) return rc;
    return execute<T>(m, (1LL << 40) | n, seq, stream);
}

template <typename T>
int do_step_backward(gsim_model* m, const gsim_params* p, gsim_state s, gsim_state ap, gsim_state am,
                     const gsim_grads* g, void* stream) {
    if (!s.x || !s.v || !ap.x || !ap.v || !am.x || !am.v) return fail(GSIM_E_INVALID, "NULL state");
    if (ap.x == am.x || ap.v == am.v) return fail(GSIM_E_INVALID, "adj_plus and adj_minus must not alias");
    int rc = check_params(m, p, g);
    if (rc) return rc;
    std::vector<StepDev<T>> rows(1);
    std::memset(rows.data(), 0, sizeof(StepDev<T>));
    StepDev<T>& r = rows[0];
    fill_params<T>(r, p, g);
    r.x = (const T*)s.x;
    r.v = (const T*)s.v;
    r.x_abs = 1;
    r.xb = (const T*)ap.x;
    r.vb = (const T*)ap.v;
    r.xbo = (T*)am.x;
    r.vbo = (T*)am.v;
    r.nsteps = 1;
    r.ckpt_every = m->K;
    r.adj = 1;
    const int64_t r0 = region_misc(m);
    if ((rc = upload_rows<T>(m, r0, rows, stream))) return rc;
    if (m->exec == GSIM_EXEC_FUSED) {
        const bool act = g && (g->act || g->hact);
        std::vector<Launch> fseq{{OP_FUSED_PARAMS, r0}, {act ? OP_FUSED_ADJ_ACT : OP_FUSED_ADJ, r0}, {OP_FUSED_GRADS, r0}};
        return execute<T>(m, (9LL << 40) | (act ? 1 : 0), fseq, stream);
    }
    std::vector<Launch> seq;
    if (g && g->contact) seq.push_back({OP_FILL_CPART, r0});
    seq.push_back({OP_ADJ, r0});
    if (g && g->contact) seq.push_back({OP_CONTACT_REDUCE, r0});
    return execute<T>(m, (2LL << 40) | (g && g->contact ? 1 : 0), seq, stream);
}

template <typename T>
int do_rollout(gsim_model* m, const gsim_params* p, gsim_state s0, int n, void* ckpt, gsim_state sf, void* stream) {
    if (n < 1 || n > m->max_steps) return fail(GSIM_E_INVALID, "n_steps must be in [1, %d]", m->max_steps);
    if (!s0.x || !s0.v || !sf.x || !sf.v) return fail(GSIM_E_INVALID, "NULL state");
    int rc = check_params(m, p);
    if (rc) return rc;
    if (ckpt) m->tail_ckpt = nullptr;  // new checkpoints: any kept segment is stale
    if (m->exec == GSIM_EXEC_FUSED)
        return do_fused_forward<T>(m, p, (const T*)s0.x, (const T*)s0.v, (T*)sf.x, (T*)sf.v, (T*)ckpt, n,
                                   region_rollout(m), (6LL << 40) | ((long long)n << 1) | (ckpt ? 1 : 0), stream);
    Ctx<T> c = ctx<T>(m);
    const int64_t S = 6 * c.np;
    // With the second segment buffer, the states of the last checkpoint segment (steps
    // tl0 + 1 .. n - 1) go there instead of the ping-pong buffers: the backward that
    // follows finds them in place of its first recompute (same steps, same inputs).
    const bool tail = ckpt && uses_seg2(m);
    const int tl0 = (n - 1) / m->K * m->K;
    auto state = [&](int t) -> T* {  // where step t - 1 leaves state t (0 < t < n)
        return tail && t > tl0 ? (T*)m->seg2 + (int64_t)(t - tl0 - 1) * S : c.fbuf + ((t - 1) & 1) * S;
    };
    std::vector<StepDev<T>> rows(n);
    std::vector<Launch> seq;
    for (int t = 0; t < n; ++t) {
        StepDev<T>& r = rows[t];
        std::memset(&r, 0, sizeof r);
        fill_params<T>(r, p, nullptr);
        at_step<T>(r, p, nullptr, t);
        if (t == 0) {
            r.x = (const T*)s0.x;
            r.v = (const T*)s0.v;
            r.x_abs = 1;
        } else {
            r.x = state(t);
            r.v = r.x + 3 * c.np;
        }
        if (t == n - 1) {
            r.xo = (T*)sf.x;
            r.vo = (T*)sf.v;
            r.xo_abs = 1;
        } else {
            r.xo = state(t + 1);
            r.vo = r.xo + 3 * c.np;
        }
        if (ckpt && t % m->K == 0) {
            r.ckx = (T*)ckpt + (int64_t)(t / m->K) * S;
            r.ckv = r.ckx + 3 * c.np;
        }
        seq.push_back({OP_FWD, region_rollout(m) + t});
    }
    if ((rc = upload_rows<T>(m, region_rollout(m), rows, stream))) return rc;
    if ((rc = execute<T>(m, (3LL << 40) | ((long long)n << 1) | (ckpt ? 1 : 0), seq, stream))) return rc;
    if (tail) {
        m->tail_ckpt = ckpt;
        m->tail_seg2 = m->seg2;
        m->tail_n = n;
    }
    return GSIM_OK;
}

template <typename T>
int do_rollout_backward(gsim_model* m, const gsim_params* p, const void* ckpt, int n, void* seg, gsim_state af,
                        gsim_state ai, const gsim_grads* g, void* stream) {
    if (n < 1 || n > m->max_steps) return fail(GSIM_E_INVALID, "n_steps must be in [1, %d]", m->max_steps);
    if (!ckpt || !seg) return fail(GSIM_E_INVALID, "checkpoint and segment buffers are required");
    if (!af.x || !af.v || !ai.x || !ai.v) return fail(GSIM_E_INVALID, "NULL adjoint state");
    int rc = check_params(m, p, g);
    if (rc) return rc;
    if (m->exec == GSIM_EXEC_FUSED)
        return do_fused_rollout_backward<T>(m, p, (const T*)ckpt, n, (T*)seg, af, ai, g, stream);
    Ctx<T> c = ctx<T>(m);
    const int64_t S = 6 * c.np, np = c.np;
    const int K = m->K;
    const int nseg = (n + K - 1) / K;
    std::vector<StepDev<T>> rows;
    std::vector<Launch> seq;
    const int64_t r0 = region_backward(m);
    const bool want_contact = g && g->contact;
    StepDev<T> base;
    std::memset(&base, 0, sizeof base);
    fill_params<T>(base, p, g);
    if (want_contact) {
        rows.push_back(base);
        seq.push_back({OP_FILL_CPART, r0});
    }
    const T* ck = (const T*)ckpt;
    T* fbar = (T*)(m->ws + m->L.fbar);
    // Overlapped recompute: with the second segment buffer (gsim_model_set_overlap), the
    // last segment's states live there and the others alternate between the caller's
    // buffer and it, and the recompute of segment s - 1 runs in the same launches as
    // segment s's adjoint steps.  When the rollout of these checkpoints left the last
    // segment's states in that buffer, that segment is not recomputed.
    const bool two = uses_seg2(m), overlap = two && nseg > 1 && m->exec != GSIM_EXEC_PERSIST;
    const bool kept = two && m->tail_ckpt == ckpt && m->tail_seg2 == m->seg2 && m->tail_n == n;
    m->tail_ckpt = nullptr;  // this call overwrites the second buffer
    auto segbuf = [&](int s) -> T* { return two && ((nseg - 1 - s) & 1) == 0 ? (T*)m->seg2 : (T*)seg; };
    std::vector<std::vector<int64_t>> rec(nseg), adj(nseg);  // table rows of each segment's passes
    int q = 0;  // adjoint steps done
    for (int s = nseg - 1; s >= 0; --s) {
        const int t0 = s * K, t1 = std::min(n, t0 + K), L = t1 - t0;
        T* segT = segbuf(s);
        // recompute states t0+1 .. t1-1 into seg[0 .. L-2]
        for (int j = 0; j + 1 < L && !(kept && s == nseg - 1); ++j) {
            StepDev<T> r = base;
            r.g_mu = r.g_lam = r.g_ktri = r.g_mass = r.g_contact = r.g_act = r.g_hact = nullptr;
            at_step<T>(r, p, nullptr, t0 + j);
            r.x = j == 0 ? ck + s * S : segT + (j - 1) * S;
            r.v = r.x + 3 * np;
            r.xo = segT + j * S;
            r.vo = r.xo + 3 * np;
            rows.push_back(r);
            rec[s].push_back(r0 + (int64_t)rows.size() - 1);
        }
        for (int t = t1 - 1; t >= t0; --t, ++q) {
            StepDev<T> r = base;
            at_step<T>(r, p, g, t);
            r.x = t == t0 ? ck + s * S : segT + (t - t0 - 1) * S;
            r.v = r.x + 3 * np;
            if (q == 0) {
                r.xb = (const T*)af.x;
                r.vb = (const T*)af.v;
            } else {
                r.xb = c.abuf + ((q - 1) & 1) * S;
                r.vb = r.xb + 3 * np;
            }
            if (t == 0) {
                r.xbo = (T*)ai.x;
                r.vbo = (T*)ai.v;
            } else {
                r.xbo = c.abuf + (q & 1) * S;
                r.vbo = r.xbo + 3 * np;
                r.fbo = fbar + (q & 1) * 3 * np;  // this step hands step t-1 its adjoint force
            }
            if (q > 0) r.fb = fbar + ((q - 1) & 1) * 3 * np;
            r.adj = 1;
            rows.push_back(r);
            adj[s].push_back(r0 + (int64_t)rows.size() - 1);
        }
    }
    if (!overlap) {
        for (int s = nseg - 1; s >= 0; --s) {
            for (int64_t row : rec[s]) seq.push_back({OP_FWD, row});
            for (int64_t row : adj[s]) seq.push_back({OP_ADJ, row});
        }
    } else {
        // the last segment's recompute alone, then each segment's adjoint steps paired
        // with the previous segment's recompute steps (two independent chains)
        for (int64_t row : rec[nseg - 1]) seq.push_back({OP_FWD, row});
        for (int s = nseg - 1; s >= 0; --s) {
            const std::vector<int64_t>& A = adj[s];
            static const std::vector<int64_t> none;
            const std::vector<int64_t>& R = s > 0 ? rec[s - 1] : none;
            const size_t k = std::min(A.size(), R.size());
            for (size_t i = 0; i < k; ++i) seq.push_back({OP_DUAL, A[i], R[i]});
            for (size_t i = k; i < A.size(); ++i) seq.push_back({OP_ADJ, A[i]});
            for (size_t i = k; i < R.size(); ++i) seq.push_back({OP_FWD, R[i]});
        }
    }
    if (want_contact) seq.push_back({OP_CONTACT_REDUCE, r0});
    if ((rc = upload_rows<T>(m, r0, rows, stream))) return rc;
    return execute<T>(m, (4LL << 40) | (overlap ? 1LL << 39 : 0) | (kept ? 1LL << 38 : 0) | (two ? 1LL << 37 : 0) |
                             ((long long)n << 1) | (want_contact ? 1 : 0),
                      seq, stream);
}

template <typename T>
int do_loss(gsim_model* m, gsim_state s, const void* target, void* loss, gsim_state adj, void* stream) {
    if (!s.x || !target || !loss) return fail(GSIM_E_INVALID, "NULL argument");
    std::vector<StepDev<T>> rows(1);
    std::memset(rows.data(), 0, sizeof(StepDev<T>));
    rows[0].x = (const T*)s.x;
    rows[0].x_abs = 1;
    rows[0].target = (const T*)target;
    rows[0].loss = (T*)loss;
    rows[0].xbo = (T*)adj.x;
    rows[0].vbo = (T*)adj.v;
    const int64_t r0 = region_misc(m) + 1;
    int rc = upload_rows<T>(m, r0, rows, stream);
    if (rc) return rc;
    std::vector<Launch> seq{{OP_LOSS, r0}};
    return execute<T>(m, 5LL << 40, seq, stream);
}

template <typename T, typename F>
int guarded(F f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return fail(GSIM_E_INVALID, "out of host memory");
    } catch (...) {
        return fail(GSIM_E_INVALID, "internal error");
    }
}

}  // namespace

namespace gsim {

template <typename T>
int model_init(const gsim_plan* P, int max_steps, int K, void* d_ws, size_t bytes, void* stream, gsim_model** out,
               UploadSink* sink) {
    Layout L = make_layout<T>(P, max_steps);
    if (bytes < L.total) return fail(GSIM_E_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, L.total);
    if (((uintptr_t)d_ws & 255) != 0) return fail(GSIM_E_INVALID, "workspace must be 256-byte aligned");
    gsim_model* m = new (std::nothrow) gsim_model();
    if (!m) return fail(GSIM_E_INVALID, "out of host memory");
    m->dtype = P->dtype;
    m->nb = P->nb;
    m->np = P->np;
    m->ne = P->ne;
    m->nt = P->nt;
    m->nh = P->nh;
    m->max_steps = max_steps;
    m->K = K;
    m->ws = (char*)d_ws;
    m->L = L;
    m->poff = P->poff;
    m->eoff = P->eoff;
    m->toff = P->toff;
    m->hoff = P->hoff;
    hipStream_t s = (hipStream_t)stream;
    char* ws = m->ws;
    auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return sink ? sink->copy(ws + off, src, n) : hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, s);
    };
    auto cvt = [](const std::vector<double>& v) { return std::vector<T>(v.begin(), v.end()); };
    std::vector<T> tet_dinv = cvt(P->tet_dinv), tet_vol = cvt(P->tet_vol), tri_dinv = cvt(P->tri_dinv),
                   tri_area = cvt(P->tri_area), hin_phi0 = cvt(P->hin_phi0);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    chk(up(L.tet_code, P->tet_code.data(), P->tet_code.size() * 4));
    chk(up(L.tet_dinv, tet_dinv.data(), tet_dinv.size() * sizeof(T)));
    chk(up(L.tet_vol, tet_vol.data(), tet_vol.size() * sizeof(T)));
    chk(up(L.tri_code, P->tri_code.data(), P->tri_code.size() * 4));
    chk(up(L.tri_dinv, tri_dinv.data(), tri_dinv.size() * sizeof(T)));
    chk(up(L.tri_area, tri_area.data(), tri_area.size() * sizeof(T)));
    chk(up(L.hin_code, P->hin_code.data(), P->hin_code.size() * 4));
    chk(up(L.hin_phi0, hin_phi0.data(), hin_phi0.size() * sizeof(T)));
    std::vector<int32_t> tp3(3 * P->tp_id.size(), 0);
    for (size_t i = 0; i < P->tp_id.size(); ++i) {
        tp3[3 * i] = P->tp_id[i];
        tp3[3 * i + 1] = P->tp_run[i];
        tp3[3 * i + 2] = P->tp_slot[i];
    }
    chk(up(L.tp, tp3.data(), tp3.size() * 4));
    chk(up(L.gbase, P->gbase.data(), P->gbase.size() * 4));
    chk(up(L.pdeg, P->pdeg.data(), P->pdeg.size() * 4));
    chk(up(L.pinned, P->pinned.data(), P->pinned.size()));
    // rest positions (SoA) and each particle's rest gap to its body's ground plane,
    // n.X - d, formed in FP64 and rounded once
    std::vector<T> rest(3 * P->np), rgap(P->np);
    for (int b = 0; b < P->nb; ++b)
        for (int64_t i = P->poff[b]; i < P->poff[b + 1]; ++i) {
            const double* x = &P->rest[3 * i];
            const double* pl = &P->plane[4 * b];
            for (int c = 0; c < 3; ++c) rest[c * P->np + i] = (T)x[c];
            rgap[i] = (T)(pl[0] * x[0] + pl[1] * x[1] + pl[2] * x[2] - pl[3]);
        }
    chk(up(L.rest, rest.data(), rest.size() * sizeof(T)));
    chk(up(L.rgap, rgap.data(), rgap.size() * sizeof(T)));
    // (set-up, never inside a captured sequence)
    chk(sink ? sink->zero(ws + L.bflag, 2 * (size_t)P->nb * 4) : hipMemsetAsync(ws + L.bflag, 0, 2 * (size_t)P->nb * 4, s));
    if (P->coloured) {  // colour-ordered copies of the element records (fused path)
        // corner indices become body-local (the fused kernels address the body's particles in LDS)
        auto perm_i = [P](const std::vector<int32_t>& a, const std::vector<int32_t>& ord, int rows, int64_t n,
                          const std::vector<int64_t>& off) {
            std::vector<int32_t> out(a.size());
            for (int b = 0; b < P->nb; ++b)
                for (int r = 0; r < rows; ++r)
                    for (int64_t e = off[b]; e < off[b + 1]; ++e)
                        out[r * n + e] = (int32_t)(a[r * n + ord[e]] - P->poff[b]);
            return out;
        };
        auto perm_t = [](const std::vector<T>& a, const std::vector<int32_t>& ord, int rows, int64_t n) {
            std::vector<T> out(a.size());
            for (int r = 0; r < rows; ++r)
                for (int64_t e = 0; e < n; ++e) out[r * n + e] = a[r * n + ord[e]];
            return out;
        };
        std::vector<int32_t> f_tet_idx = perm_i(P->tet_idx, P->ftet, 4, P->ne, P->eoff),
                             f_tri_idx = perm_i(P->tri_idx, P->ftri, 3, P->nt, P->toff),
                             f_hin_idx = perm_i(P->hin_idx, P->fhin, 4, P->nh, P->hoff);
        std::vector<T> f_tet_dinv = perm_t(tet_dinv, P->ftet, 9, P->ne), f_tet_vol = perm_t(tet_vol, P->ftet, 1, P->ne),
                       f_tri_dinv = perm_t(tri_dinv, P->ftri, 4, P->nt), f_tri_area = perm_t(tri_area, P->ftri, 1, P->nt),
                       f_hin_phi0 = perm_t(hin_phi0, P->fhin, 1, P->nh);
        chk(up(L.f_tet_idx, f_tet_idx.data(), f_tet_idx.size() * 4));
        chk(up(L.f_tet_dinv, f_tet_dinv.data(), f_tet_dinv.size() * sizeof(T)));
        chk(up(L.f_tet_vol, f_tet_vol.data(), f_tet_vol.size() * sizeof(T)));
        chk(up(L.f_tet_orig, P->ftet.data(), P->ftet.size() * 4));
        chk(up(L.f_tri_idx, f_tri_idx.data(), f_tri_idx.size() * 4));
        chk(up(L.f_tri_dinv, f_tri_dinv.data(), f_tri_dinv.size() * sizeof(T)));
        chk(up(L.f_tri_area, f_tri_area.data(), f_tri_area.size() * sizeof(T)));
        chk(up(L.f_tri_orig, P->ftri.data(), P->ftri.size() * 4));
        chk(up(L.f_hin_idx, f_hin_idx.data(), f_hin_idx.size() * 4));
        chk(up(L.f_hin_phi0, f_hin_phi0.data(), f_hin_phi0.size() * sizeof(T)));
        chk(up(L.f_hin_orig, P->fhin.data(), P->fhin.size() * 4));
        chk(up(L.coff, P->coff.data(), P->coff.size() * 4));
    }
    // fused launch order: largest bodies first (they bound the makespan)
    std::vector<int32_t> border(P->nb);
    for (int b = 0; b < P->nb; ++b) border[b] = b;
    std::stable_sort(border.begin(), border.end(), [&](int32_t a, int32_t c) {
        const int64_t wa = (P->eoff[a + 1] - P->eoff[a]) + (P->toff[a + 1] - P->toff[a]) + (P->hoff[a + 1] - P->hoff[a]);
        const int64_t wc = (P->eoff[c + 1] - P->eoff[c]) + (P->toff[c + 1] - P->toff[c]) + (P->hoff[c + 1] - P->hoff[c]);
        return wa > wc;
    });
    chk(up(L.border, border.data(), border.size() * 4));
    m->fused_ok = P->fused_ok;
    m->any_air = P->any_air;
    m->air_on = P->air_on;
    m->etiles_plan = P->etiles;
    m->etile_words[0] = P->etile_words[0];
    m->etile_words[1] = P->etile_words[1];
    // fused dynamic LDS of a body: its particle arrays, then its colour bounds (int32,
    // ncol + 1 per element kind)
    for (int b = 0; b < P->nb; ++b) {
        const int64_t npb = P->poff[b + 1] - P->poff[b];
        const size_t cbb = 4 * (size_t)(P->ncol[3 * b] + P->ncol[3 * b + 1] + P->ncol[3 * b + 2] + 3);
        m->max_body_np = std::max<int64_t>(m->max_body_np, npb);
        m->fused_dyn[0] = std::max(m->fused_dyn[0], FUSED_FWD_LDS_WORDS * sizeof(T) * (size_t)npb + cbb);
        m->fused_dyn[1] = std::max(m->fused_dyn[1], FUSED_ADJ_LDS_WORDS * sizeof(T) * (size_t)npb + cbb);
    }
    std::vector<BodyDev<T>> bodies(P->nb);
    for (int b = 0; b < P->nb; ++b) {
        BodyDev<T>& B = bodies[b];
        std::memset(&B, 0, sizeof B);
        B.p0 = P->poff[b];
        B.np = P->poff[b + 1] - P->poff[b];
        B.contact_on = P->contact_on[b];
        B.air_on = P->air_on[b];
        B.g0 = P->body_g0[b];
        for (int k = 0; k < 3; ++k) {
            B.cbase[k] = P->cbase[3 * b + k];
            B.ncol[k] = P->ncol[3 * b + k];
        }
        B.dt = (T)P->dt[b];
        for (int c = 0; c < 3; ++c) B.g[c] = (T)P->grav[3 * b + c];
        for (int c = 0; c < 4; ++c) B.plane[c] = (T)P->plane[4 * b + c];
        B.kb = (T)P->kb[b];
    }
    m->bodies_host.assign(reinterpret_cast<const char*>(bodies.data()),
                          reinterpret_cast<const char*>(bodies.data() + P->nb));
    ModelDev<T> M;
    std::memset(&M, 0, sizeof M);
    M.np = P->np;
    M.ne = P->ne;
    M.nt = P->nt;
    M.nh = P->nh;
    M.nslot = P->nslot;
    M.n_bodies = P->nb;
    M.tet_code = (const uint32_t*)(ws + L.tet_code);
    M.tet_dinv = (const T*)(ws + L.tet_dinv);
    M.tet_vol = (const T*)(ws + L.tet_vol);
    M.tri_code = (const uint32_t*)(ws + L.tri_code);
    M.tri_dinv = (const T*)(ws + L.tri_dinv);
    M.tri_area = (const T*)(ws + L.tri_area);
    M.hin_code = (const uint32_t*)(ws + L.hin_code);
    M.hin_phi0 = (const T*)(ws + L.hin_phi0);
    M.tp = (const int32_t*)(ws + L.tp);
    M.gbase = (const int32_t*)(ws + L.gbase);
    M.pdeg = (const int32_t*)(ws + L.pdeg);
    M.pinned = (const uint8_t*)(ws + L.pinned);
    M.rest = (const T*)(ws + L.rest);
    M.rgap = (const T*)(ws + L.rgap);
    M.bflag = (int32_t*)(ws + L.bflag);
    M.bodies = (const BodyDev<T>*)(ws + L.bodies);
    M.slots = (T*)(ws + L.slots);
    M.fslots = (T*)(ws + L.fslots);
    M.vslots = P->any_air ? (T*)(ws + L.vslots) : nullptr;
    M.cpart = (T*)(ws + L.cpart);
    M.lpart = (T*)(ws + L.lpart);
    M.f_tet_idx = (const int32_t*)(ws + L.f_tet_idx);
    M.f_tet_dinv = (const T*)(ws + L.f_tet_dinv);
    M.f_tet_vol = (const T*)(ws + L.f_tet_vol);
    M.f_tet_orig = (const int32_t*)(ws + L.f_tet_orig);
    M.f_tri_idx = (const int32_t*)(ws + L.f_tri_idx);
    M.f_tri_dinv = (const T*)(ws + L.f_tri_dinv);
    M.f_tri_area = (const T*)(ws + L.f_tri_area);
    M.f_tri_orig = (const int32_t*)(ws + L.f_tri_orig);
    M.f_hin_idx = (const int32_t*)(ws + L.f_hin_idx);
    M.f_hin_phi0 = (const T*)(ws + L.f_hin_phi0);
    M.f_hin_orig = (const int32_t*)(ws + L.f_hin_orig);
    M.coff = (const int32_t*)(ws + L.coff);
    M.f_par = (T*)(ws + L.f_par);
    M.f_ktri = (T*)(ws + L.f_ktri);
    M.f_g = (T*)(ws + L.f_g);
    M.f_gk = (T*)(ws + L.f_gk);
    M.f_hpar = (T*)(ws + L.f_hpar);
    M.f_gh = (T*)(ws + L.f_gh);
    chk(up(L.model, &M, sizeof M));
    m->md_host.assign(reinterpret_cast<const char*>(&M), reinterpret_cast<const char*>(&M) + sizeof M);
    chk(hipEventCreateWithFlags(&m->stage_evt, hipEventDisableTiming));
    if (P->nb >= 2) {  // launch lanes' streams and fork / join events
        chk(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
        for (int l = 1; l < MAX_LANES; ++l) {
            chk(hipStreamCreateWithFlags(&m->lane_stream[l], hipStreamNonBlocking));
            chk(hipEventCreateWithFlags(&m->ev_join[l], hipEventDisableTiming));
        }
        m->lanes = std::min(DEFAULT_LANES, P->nb);
    }
    if (e != hipSuccess) {
        if (m->stage) (void)hipHostFree(m->stage);
        if (m->stage_evt) (void)hipEventDestroy(m->stage_evt);
        if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
        for (int l = 1; l < MAX_LANES; ++l) {
            if (m->ev_join[l]) (void)hipEventDestroy(m->ev_join[l]);
            if (m->lane_stream[l]) (void)hipStreamDestroy(m->lane_stream[l]);
        }
        delete m;
        return hip_fail(e, "upload model");
    }
    int rc = upload_tiles<T>(m, stream, sink);
    if (rc) {
        gsim_model_destroy(m);
        return rc;
    }
    *out = m;
    return GSIM_OK;
}

template int model_init<float>(const gsim_plan*, int, int, void*, size_t, void*, gsim_model**, UploadSink*);
template int model_init<double>(const gsim_plan*, int, int, void*, size_t, void*, gsim_model**, UploadSink*);

}  // namespace gsim

// ------------------------------------------------------------------ C-ABI ---
extern "C" {

const char* gsim_last_error(void) { return g_err.c_str(); }

int gsim_version(int* major, int* minor) {
    if (major) *major = 0;
    if (minor) *minor = 1;
    return GSIM_OK;
}

int gsim_plan_create(const gsim_model_desc* desc, gsim_plan** out) { return plan_create(desc, out, true); }

}  // extern "C"

int gsim::plan_create(const gsim_model_desc* desc, gsim_plan** out, bool fused) {
    if (!out) return fail(GSIM_E_INVALID, "NULL output");
    *out = nullptr;
    return guarded<double>([&]() {
        gsim_plan* P = new gsim_plan();
        int rc = build_plan(desc, P, fused);
        if (rc) {
            delete P;
            return rc;
        }
        *out = P;
        return (int)GSIM_OK;
    });
}

extern "C" {

int gsim_plan_destroy(gsim_plan* plan) {
    delete plan;
    return GSIM_OK;
}

int gsim_plan_colouring(const gsim_plan* P, int kind, int32_t* order, int32_t* bounds, int max_bounds, int* n_bounds) {
    if (!P || kind < 0 || kind > 2) return fail(GSIM_E_INVALID, "bad plan or kind");
    if (!P->fused_ok) return fail(GSIM_E_UNSUPPORTED, "colouring failed");
    const std::vector<int32_t>& ord = kind == 0 ? P->ftet : kind == 1 ? P->ftri : P->fhin;
    if (order) std::copy(ord.begin(), ord.end(), order);
    int n = 0;
    for (int b = 0; b < P->nb; ++b) {
        const int base = P->cbase[3 * b + kind], nc = P->ncol[3 * b + kind];
        for (int c = 0; c <= nc; ++c, ++n)
            if (bounds && n < max_bounds) bounds[n] = P->coff[base + c];
    }
    if (n_bounds) *n_bounds = n;
    return n <= max_bounds || !bounds ? GSIM_OK : fail(GSIM_E_WORKSPACE, "bounds array too small (%d needed)", n);
}

int gsim_plan_tiles(const gsim_plan* P, int64_t* tiles, int64_t* n_tiles, int32_t* tile_particles, int32_t* runs,
                    int32_t* slots, int64_t* n_tile_particles) {
    if (!P) return fail(GSIM_E_INVALID, "NULL plan");
    if (tiles)
        for (size_t i = 0; i < P->etiles.size(); ++i) {
            const Tile& t = P->etiles[i];
            int64_t* r = tiles + 5 * i;
            r[0] = t.kind;
            r[1] = t.body;
            r[2] = t.begin;
            r[3] = t.count;
            r[4] = t.id;
        }
    if (n_tiles) *n_tiles = (int64_t)P->etiles.size();
    if (tile_particles) std::copy(P->tp_id.begin(), P->tp_id.end(), tile_particles);
    if (runs) std::copy(P->tp_run.begin(), P->tp_run.end(), runs);
    if (slots) std::copy(P->tp_slot.begin(), P->tp_slot.end(), slots);
    if (n_tile_particles) *n_tile_particles = (int64_t)P->tp_id.size();
    return GSIM_OK;
}

int gsim_plan_codes(const gsim_plan* P, int kind, uint32_t* codes) {
    if (!P || kind < 0 || kind > 2) return fail(GSIM_E_INVALID, "bad plan or kind");
    const std::vector<uint32_t>& c = kind == 0 ? P->tet_code : kind == 1 ? P->tri_code : P->hin_code;
    if (codes) std::copy(c.begin(), c.end(), codes);
    return GSIM_OK;
}

int gsim_plan_partials(const gsim_plan* P, int32_t* slice_base, int64_t* n_slices, int32_t* degree, int64_t* n_slots) {
    if (!P) return fail(GSIM_E_INVALID, "NULL plan");
    if (slice_base) std::copy(P->gbase.begin(), P->gbase.end(), slice_base);
    if (n_slices) *n_slices = (int64_t)P->gbase.size();
    if (degree) std::copy(P->pdeg.begin(), P->pdeg.end(), degree);
    if (n_slots) *n_slots = P->nslot;
    return GSIM_OK;
}

int gsim_plan_counts(const gsim_plan* P, int64_t* np, int64_t* ne, int64_t* nt, int64_t* nh, int* nb) {
    if (!P) return fail(GSIM_E_INVALID, "NULL plan");
    if (np) *np = P->np;
    if (ne) *ne = P->ne;
    if (nt) *nt = P->nt;
    if (nh) *nh = P->nh;
    if (nb) *nb = P->nb;
    return GSIM_OK;
}

int gsim_plan_sizes(const gsim_plan* P, int max_steps, int K, size_t* ws, size_t* ck, size_t* seg) {
    if (!P) return fail(GSIM_E_INVALID, "NULL plan");
    if (max_steps < 1 || K < 1) return fail(GSIM_E_INVALID, "max_steps and ckpt_every must be >= 1");
    const size_t sz = P->dtype == GSIM_F64 ? 8 : 4;
    const size_t state = 6 * (size_t)P->np * sz;
    if (ws) *ws = P->dtype == GSIM_F64 ? make_layout<double>(P, max_steps).total : make_layout<float>(P, max_steps).total;
    if (ck) *ck = (size_t)((max_steps + K - 1) / K) * state;
    if (seg) *seg = (size_t)K * state;
    return GSIM_OK;
}

int gsim_model_init(const gsim_plan* P, int max_steps, int K, void* d_ws, size_t bytes, void* stream, gsim_model** out) {
    if (!P || !out || !d_ws) return fail(GSIM_E_INVALID, "NULL argument");
    if (max_steps < 1 || K < 1) return fail(GSIM_E_INVALID, "max_steps and ckpt_every must be >= 1");
    *out = nullptr;
    return guarded<double>([&]() {
        return P->dtype == GSIM_F64 ? model_init<double>(P, max_steps, K, d_ws, bytes, stream, out)
                                    : model_init<float>(P, max_steps, K, d_ws, bytes, stream, out);
    });
}

int gsim_model_destroy(gsim_model* m) {
    if (!m) return GSIM_OK;
    for (auto& g : m->graphs)
        if (g.second.exec) (void)hipGraphExecDestroy(g.second.exec);
    if (m->stage_evt) {
        (void)hipEventSynchronize(m->stage_evt);
        (void)hipEventDestroy(m->stage_evt);
    }
    if (m->stage) (void)hipHostFree(m->stage);
    for (int l = 1; l < MAX_LANES; ++l) {
        if (m->lane_stream[l]) {
            (void)hipStreamSynchronize(m->lane_stream[l]);
            (void)hipStreamDestroy(m->lane_stream[l]);
        }
        if (m->ev_join[l]) (void)hipEventDestroy(m->ev_join[l]);
    }
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    for (auto& p : m->pending) {
        (void)hipEventSynchronize(p.b);
        m->evt_pool.push_back(p.a);
        m->evt_pool.push_back(p.b);
    }
    for (hipEvent_t e : m->evt_pool) (void)hipEventDestroy(e);
    delete m;
    return GSIM_OK;
}

int gsim_model_set_launch(gsim_model* m, int pass, int block, int items) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (pass != 0 && pass != 1) return fail(GSIM_E_INVALID, "pass must be 0 (element) or 1 (particle)");
    if (block < 64 || block > 512 || block % 64) return fail(GSIM_E_INVALID, "block must be 64..512, multiple of 64");
    if (items < 1 || items > 8) return fail(GSIM_E_INVALID, "items must be 1..8");
    int& b = pass == 0 ? m->block : m->pblock;
    int& i = pass == 0 ? m->items : m->pitems;
    if (b == block && i == items) return GSIM_OK;
    // the tile lists are rewritten in place: wait until no launch can still read them
    HIP_TRY(hipDeviceSynchronize(), "synchronize before retiling");
    b = block;
    i = items;
    return guarded<double>([&]() { return m->dtype == GSIM_F64 ? upload_tiles<double>(m, nullptr) : upload_tiles<float>(m, nullptr); });
}

int gsim_model_set_lanes(gsim_model* m, int lanes) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (lanes < 1 || lanes > MAX_LANES) return fail(GSIM_E_INVALID, "lanes must be 1..%d", MAX_LANES);
    if (lanes > m->nb) return fail(GSIM_E_UNSUPPORTED, "%d lanes need at least %d bodies", lanes, lanes);
    if (m->lanes == lanes) return GSIM_OK;
    HIP_TRY(hipDeviceSynchronize(), "synchronize before retiling");
    m->lanes = lanes;
    return guarded<double>([&]() { return m->dtype == GSIM_F64 ? upload_tiles<double>(m, nullptr) : upload_tiles<float>(m, nullptr); });
}

int gsim_model_set_overlap(gsim_model* m, void* d_segment2, size_t bytes) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    m->tail_ckpt = nullptr;
    if (!d_segment2) {
        m->seg2 = nullptr;
        m->seg2_bytes = 0;
        return GSIM_OK;
    }
    const size_t need = (size_t)std::max(m->K - 1, 1) * 6 * (size_t)m->np * (m->dtype == GSIM_F64 ? 8 : 4);
    if (bytes < need) return fail(GSIM_E_WORKSPACE, "second segment buffer: %zu bytes, need %zu", bytes, need);
    m->seg2 = d_segment2;
    m->seg2_bytes = bytes;
    return GSIM_OK;
}

int gsim_model_get_lanes(const gsim_model* m, int* lanes) {
    if (!m || !lanes) return fail(GSIM_E_INVALID, "NULL argument");
    *lanes = m->lanes;
    return GSIM_OK;
}

int gsim_model_get_launch(const gsim_model* m, int pass, int* block, int* items) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (pass != 0 && pass != 1) return fail(GSIM_E_INVALID, "pass must be 0 (element) or 1 (particle)");
    if (block) *block = pass == 0 ? m->block : m->pblock;
    if (items) *items = pass == 0 ? m->items : m->pitems;
    return GSIM_OK;
}

int gsim_model_set_exec(gsim_model* m, int exec, int block, int items) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (exec != GSIM_EXEC_PLAIN && exec != GSIM_EXEC_GRAPH && exec != GSIM_EXEC_FUSED && exec != GSIM_EXEC_PERSIST)
        return fail(GSIM_E_INVALID, "unknown exec %d", exec);
    if (exec == GSIM_EXEC_PERSIST && m->any_air)
        return fail(GSIM_E_UNSUPPORTED, "persistent execution does not model lift/drag (a body has air_on)");
    if (exec == GSIM_EXEC_PERSIST && m->dtype != GSIM_F32)
        return fail(GSIM_E_UNSUPPORTED, "persistent execution is FP32 only");
    if (exec == GSIM_EXEC_FUSED) {
        if (!m->fused_ok) return fail(GSIM_E_UNSUPPORTED, "fused execution: an element kind needs more than 128 colours");
        if (m->any_air) return fail(GSIM_E_UNSUPPORTED, "fused execution does not model lift/drag (a body has air_on)");
        int dev = 0, lds_max = 0;
        HIP_TRY(hipGetDevice(&dev), "get device");
        HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "device LDS size");
        // each kernel's static LDS (colour bounds, block reduction) + its dynamic LDS
        size_t st_f = 0, st_a = 0, need = 0;
        const bool f64 = m->dtype == GSIM_F64;
        HIP_TRY(f64 ? fused_static_lds<double>(false, &st_f) : fused_static_lds<float>(false, &st_f), "fused LDS size");
        HIP_TRY(f64 ? fused_static_lds<double>(true, &st_a) : fused_static_lds<float>(true, &st_a), "fused LDS size");
        need = f64 ? std::max(st_f + fused_lds<double>(m, false), st_a + fused_lds<double>(m, true))
                   : std::max(st_f + fused_lds<float>(m, false), st_a + fused_lds<float>(m, true));
        if (need > (size_t)lds_max)
            return fail(GSIM_E_UNSUPPORTED, "fused execution: the largest body needs %zu bytes of LDS, the device has %d",
                        need, lds_max);
    }
    if (block && (block < 64 || block > 512 || block % 64)) return fail(GSIM_E_INVALID, "block must be 64..512, multiple of 64");
    if (items && (items < 1 || items > 8)) return fail(GSIM_E_INVALID, "items must be 1..8");
    m->exec = exec;
    for (int pass = 0; pass < 2; ++pass) {
        int b = 0, i = 0;
        gsim_model_get_launch(m, pass, &b, &i);
        int rc = gsim_model_set_launch(m, pass, block ? block : b, items ? items : i);
        if (rc) return rc;
    }
    return GSIM_OK;
}

int gsim_model_get_exec(const gsim_model* m, int* exec, int* block, int* items) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (exec) *exec = m->exec;
    if (block) *block = m->block;
    if (items) *items = m->items;
    return GSIM_OK;
}

int gsim_model_set_timing(gsim_model* m, int mask) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (mask < 0 || mask > 255) return fail(GSIM_E_INVALID, "timing mask must be in [0, 255]");
    if (mask && m->exec == GSIM_EXEC_PERSIST) return fail(GSIM_E_UNSUPPORTED, "kernel timing needs plain execution");
    m->timing_mask = mask;
    return GSIM_OK;
}

int gsim_model_read_timing(gsim_model* m, int kernel, int64_t* launches, double* total_ms) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    if (kernel < 0 || kernel > 7) return fail(GSIM_E_INVALID, "kernel must be in [0, 7]");
    for (auto& p : m->pending) {
        HIP_TRY(hipEventSynchronize(p.b), "timing sync");
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b), "timing elapsed");
        m->timing_ms[p.kernel] += ms;
        m->timing_n[p.kernel] += 1;
        m->evt_pool.push_back(p.a);
        m->evt_pool.push_back(p.b);
    }
    m->pending.clear();
    if (launches) *launches = m->timing_n[kernel];
    if (total_ms) *total_ms = m->timing_ms[kernel];
    m->timing_n[kernel] = 0;
    m->timing_ms[kernel] = 0;
    return GSIM_OK;
}

int gsim_model_check(gsim_model* m, int32_t* body_flags, int clear, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    try {
        hipStream_t s = (hipStream_t)stream;
        std::vector<int32_t> f(2 * (size_t)m->nb);
        HIP_TRY(hipMemcpyAsync(f.data(), m->ws + m->L.bflag, f.size() * 4, hipMemcpyDeviceToHost, s), "read flags");
        HIP_TRY(hipStreamSynchronize(s), "read flags");
        if (clear) {
            HIP_TRY(hipMemsetAsync(m->ws + m->L.bflag, 0, f.size() * 4, s), "clear flags");
            HIP_TRY(hipStreamSynchronize(s), "clear flags");
        }
        int bad = -1, nbad = 0;
        for (int b = 0; b < m->nb; ++b) {
            const int32_t v = (f[2 * b] ? GSIM_FLAG_NONFINITE : 0) | (f[2 * b + 1] ? GSIM_FLAG_INVERTED : 0);
            if (body_flags) body_flags[b] = v;
            if (f[2 * b]) {
                nbad++;
                if (bad < 0) bad = b;
            }
        }
        if (nbad) return fail(GSIM_E_NONFINITE, "%d of %d bodies went non-finite (first: body %d)", nbad, m->nb, bad);
        return GSIM_OK;
    } catch (const std::bad_alloc&) {
        return fail(GSIM_E_INVALID, "out of host memory");
    }
}

#define DISPATCH(m, call) ((m)->dtype == GSIM_F64 ? call<double> : call<float>)

int gsim_step(gsim_model* m, const gsim_params* p, gsim_state in, gsim_state out, int n, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    return guarded<double>([&]() { return DISPATCH(m, do_step)(m, p, in, out, n, stream); });
}

int gsim_step_backward(gsim_model* m, const gsim_params* p, gsim_state s, gsim_state ap, gsim_state am,
                       const gsim_grads* g, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    return guarded<double>([&]() { return DISPATCH(m, do_step_backward)(m, p, s, ap, am, g, stream); });
}

int gsim_rollout(gsim_model* m, const gsim_params* p, gsim_state s0, int n, void* ckpt, gsim_state sf, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    return guarded<double>([&]() { return DISPATCH(m, do_rollout)(m, p, s0, n, ckpt, sf, stream); });
}

int gsim_rollout_backward(gsim_model* m, const gsim_params* p, const void* ckpt, int n, void* seg, gsim_state af,
                          gsim_state ai, const gsim_grads* g, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    return guarded<double>([&]() { return DISPATCH(m, do_rollout_backward)(m, p, ckpt, n, seg, af, ai, g, stream); });
}

int gsim_loss_mse(gsim_model* m, gsim_state s, const void* target, void* loss, gsim_state adj, void* stream) {
    if (!m) return fail(GSIM_E_INVALID, "NULL model");
    return guarded<double>([&]() { return DISPATCH(m, do_loss)(m, s, target, loss, adj, stream); });
}

}  // extern "C"

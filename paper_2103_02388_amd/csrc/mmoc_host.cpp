// mmoc_host.cpp -- host side of the MMOC tracer library: the C-ABI declared
// in include/mmoc.h, argument and mesh validation, the coarse-mesh tables and
// the unique DoF numbering (Sec. 2.1 and Sec. 2.3.1 grid data structure).
//
// Unique numbering.  Every sub-simplex (vertex, edge, face) of the coarse
// mesh is owned by the lowest-index macro that contains it; a lattice node
// is owned by the owner of the smallest sub-simplex that carries it (its
// support: the macro vertices with nonzero barycentric weight).  Walking the
// macros in index order and their nodes in lexicographic (I, J, K) order, a
// node gets the next unique index in its owner; elsewhere it takes the index
// of the same node in the owner, found by re-expressing its barycentric
// weights in the owner's vertex order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/mmoc.h"
#include "mmoc_ctx.h"
#include "mmoc_internal.h"

using mmoc::MacroGeo;

mmoc_status fail(mmoc_ctx* c, mmoc_status st, const char* fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return st;
}

// A failed runtime call also leaves its error as the thread's last HIP
// error, which the next launch check would report again: it is consumed here,
// once it has been returned to the caller.
mmoc_status hip_fail(mmoc_ctx* c, hipError_t e, const char* what)
{
    (void)hipGetLastError();
    return fail(c, e == hipErrorOutOfMemory ? MMOC_E_NOMEM : MMOC_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {

}  // namespace

// A device pointer must be device memory of the context's GPU, aligned, and
// its allocation must hold `bytes` from p on.
mmoc_status check_dev(mmoc_ctx* c, const void* p, size_t bytes, size_t align, const char* name)
{
    if (!p) return fail(c, MMOC_E_ARG, "%s is null", name);
    if (reinterpret_cast<uintptr_t>(p) % align) return fail(c, MMOC_E_ARG, "%s is not %zu-byte aligned", name, align);
    hipPointerAttribute_t at;
    hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, MMOC_E_ARG, "%s is not a device pointer", name);
    }
    if (at.type != hipMemoryTypeDevice) return fail(c, MMOC_E_ARG, "%s is not device memory", name);
    if (at.device != c->device) return fail(c, MMOC_E_ARG, "%s lives on device %d, context on %d", name, at.device, c->device);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, MMOC_E_ARG, "%s: allocation range unknown", name);
    }
    const char* b = reinterpret_cast<const char*>(base);
    const char* q = reinterpret_cast<const char*>(p);
    if (q < b || (size_t)(q - b) + bytes > size)
        return fail(c, MMOC_E_ARG, "%s: allocation too small (%zu bytes needed from this address)", name, bytes);
    return MMOC_OK;
}

namespace {

template <typename T>
mmoc_status dev_alloc(mmoc_ctx* c, T** p, size_t count, const char* what)
{
    *p = nullptr;
    if (count == 0) return MMOC_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(c, e, what);
    }
    return MMOC_OK;
}

mmoc_status alloc_clear(mmoc_ctx* c, void** p, size_t bytes, const char* what)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(c, e, what);
    }
    HIPCHK(c, hipMemsetAsync(*p, 0, bytes, c->stream), what);
    return MMOC_OK;
}

// (Re)allocates the ring of `levels` velocity levels; every level unset.
// The old ring is released first (the new one may need its memory).  The
// context's ring fields change only once both new arrays exist; if either
// allocation fails the context holds no levels (lev_cap 0, nothing set), so
// that every later trace call fails with MMOC_E_STATE until the level count
// is set again.
mmoc_status alloc_velocity_levels(mmoc_ctx* c, int levels)
{
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->va_all);
    (void)hipFree(c->vb_all);
    c->va_all = c->vb_all = nullptr;
    c->lev_cap = 0;
    c->rot = 0;
    c->vel_set.assign(2, 0);
    const bool f32 = c->prec != MMOC_FP64;
    const size_t elem = f32 ? sizeof(float) : sizeof(double);
    const int na = (c->dim == 3 && f32) ? 3 : 2;
    const bool split = c->dim == 3 && !f32;  // u_z in vb_all
    const int64_t lsa = c->nslots * na;
    const int zs = (split && levels == 2) ? 2 : 1;
    const int64_t lsb = split ? (zs == 2 ? 1 : c->nslots) : 0;
    void* va = nullptr;
    void* vb = nullptr;
    mmoc_status st;
    if ((st = alloc_clear(c, &va, (size_t)lsa * elem * levels, "velocity arrays")) != MMOC_OK) return st;
    if (split && (st = alloc_clear(c, &vb, (size_t)c->nslots * elem * levels, "velocity arrays")) != MMOC_OK) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(va);
        return st;
    }
    c->va_all = va;
    c->vb_all = vb;
    c->va_lstride = lsa;
    c->vb_lstride = lsb;
    c->zs = zs;
    c->lev_cap = levels;
    c->vel_set.assign(levels, 0);
    return MMOC_OK;
}

int64_t lattice_count(int dim, int m)
{
    return dim == 2 ? (int64_t)(m + 1) * (m + 2) / 2 : (int64_t)(m + 1) * (m + 2) * (m + 3) / 6;
}

int64_t lattice_index(int dim, int64_t I, int64_t J, int64_t K)
{
    return dim == 2 ? I * (I + 1) / 2 + J : I * (I + 1) * (I + 2) / 6 + J * (J + 1) / 2 + K;
}

// d x d inverse by cofactors; returns determinant
double invert(int d, const double* B, double* Bi)
{
    if (d == 2) {
        const double det = B[0] * B[3] - B[1] * B[2];
        Bi[0] = B[3] / det;
        Bi[1] = -B[1] / det;
        Bi[2] = -B[2] / det;
        Bi[3] = B[0] / det;
        return det;
    }
    double C[9];
    C[0] = B[4] * B[8] - B[5] * B[7];
    C[1] = B[5] * B[6] - B[3] * B[8];
    C[2] = B[3] * B[7] - B[4] * B[6];
    C[3] = B[2] * B[7] - B[1] * B[8];
    C[4] = B[0] * B[8] - B[2] * B[6];
    C[5] = B[1] * B[6] - B[0] * B[7];
    C[6] = B[1] * B[5] - B[2] * B[4];
    C[7] = B[2] * B[3] - B[0] * B[5];
    C[8] = B[0] * B[4] - B[1] * B[3];
    const double det = B[0] * C[0] + B[1] * C[1] + B[2] * C[2];
    // inverse = adj / det, adj[r][c] = C[c][r]
    for (int r = 0; r < 3; ++r)
        for (int cc = 0; cc < 3; ++cc) Bi[r * 3 + cc] = C[cc * 3 + r] / det;
    return det;
}

void free_all(mmoc_ctx* c);

}  // namespace

int64_t mmoc_lattice_index(int dim, int64_t I, int64_t J, int64_t K) { return lattice_index(dim, I, J, K); }

extern "C" {

void mmoc_default_options(mmoc_options* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->eps_in = 1e-12;
    o->eps32_macro = 4e-6f;
    o->eps32_micro = 0x1p-18f;  // float64 tie-break at micro faces too (0 turns it off)
    o->max_hops = 64;
    o->order = 2;
    o->elem_cache = 1;
}

mmoc_status mmoc_create(mmoc_ctx** out, int dim, int level, mmoc_precision prec, const mmoc_options* opt,
                        void* hip_stream)
{
    if (!out) return MMOC_E_ARG;
    *out = nullptr;
    if (dim != 2 && dim != 3) return MMOC_E_ARG;
    if (level < 0 || level > 10 || (dim == 3 && level > 9)) return MMOC_E_ARG;  // lattice index fits int32
    if (prec != MMOC_FP64 && prec != MMOC_FP32_MIXED && prec != MMOC_FP32_FIELDS) return MMOC_E_ARG;
    if (opt && (!(opt->eps_in >= 0) || opt->max_hops < 0 || !(opt->eps32_macro >= 0) || !(opt->eps32_micro >= 0) ||
                opt->order < 0 || opt->order > 2 || opt->elem_cache < 0 || opt->elem_cache > 1 ||
                opt->keep_chat < 0 || opt->keep_chat > 1))
        return MMOC_E_ARG;
    mmoc_ctx* c = new (std::nothrow) mmoc_ctx();
    if (!c) return MMOC_E_NOMEM;
    c->dim = dim;
    c->level = level;
    c->n = 1 << level;
    c->prec = prec;
    if (opt) c->opt = *opt;
    else mmoc_default_options(&c->opt);
    if (c->opt.order == 0) c->opt.order = 2;
    c->m = c->opt.order * c->n;  // DoF lattice: 2n for P2, n for P1
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MMOC_E_HIP;
    }
    // the allocation-free entry points' scratch array on this device
    if (mmoc::noalloc_scratch(c->device, &c->noalloc_d) != hipSuccess) {
        (void)hipGetLastError();
        c->noalloc_d = nullptr;
    }
    if (dev_alloc(c, &c->stats_d, (size_t)mmoc::ST_COUNT * mmoc::kStatSpread, "stats") != MMOC_OK ||
        hipMemset(c->stats_d, 0, sizeof(unsigned long long) * mmoc::ST_COUNT * mmoc::kStatSpread) != hipSuccess) {
        free_all(c);
        delete c;
        return MMOC_E_HIP;
    }
    *out = c;
    return MMOC_OK;
}

mmoc_status mmoc_set_stream(mmoc_ctx* c, void* hip_stream)
{
    if (!c) return MMOC_E_ARG;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return MMOC_OK;
}

mmoc_status mmoc_upload_mesh(mmoc_ctx* c, int nv, const double* vert, int nm, const int32_t* mv, mmoc_blend blend)
{
    if (!c) return MMOC_E_ARG;
    if (c->mesh_ok) return fail(c, MMOC_E_STATE, "mesh already uploaded");
    if (!vert || !mv || nv <= 0 || nm <= 0) return fail(c, MMOC_E_ARG, "empty mesh or null array");
    if (blend != MMOC_BLEND_NONE && blend != MMOC_BLEND_SHELL_RADIAL) return fail(c, MMOC_E_ARG, "unknown blend");
    if (blend == MMOC_BLEND_SHELL_RADIAL && c->m != 2 * c->n)
        return fail(c, MMOC_E_UNSUPPORTED, "P1 elements are not built for blended meshes");
    const int d = c->dim, nvm = d + 1;
    if (nm >= (1 << 27)) return fail(c, MMOC_E_ARG, "too many macros");
    const int64_t npm = lattice_count(d, c->m);
    if ((int64_t)nm * npm >= (int64_t)INT32_MAX) return fail(c, MMOC_E_ARG, "mesh too large for 32-bit slot indices");
    {
        // the gathers address records with 32-bit byte offsets
        const bool f32 = c->prec != MMOC_FP64;
        const uint64_t rec = (d == 3 && f32) ? 12 : (f32 ? 8 : 16);
        if ((uint64_t)nm * (uint64_t)npm * rec >= (1ull << 32))
            return fail(c, MMOC_E_ARG, "mesh too large: field arrays must stay below 4 GiB for 32-bit slot offsets");
    }
    for (int i = 0; i < nv * d; ++i)
        if (!std::isfinite(vert[i])) return fail(c, MMOC_E_MESH, "vertex coordinate %d is not finite", i);
    for (int M = 0; M < nm; ++M)
        for (int a = 0; a < nvm; ++a) {
            const int v = mv[M * nvm + a];
            if (v < 0 || v >= nv) return fail(c, MMOC_E_MESH, "macro %d vertex %d out of range", M, a);
            for (int b = 0; b < a; ++b)
                if (mv[M * nvm + b] == v) return fail(c, MMOC_E_MESH, "macro %d repeats vertex %d", M, v);
        }

    // --- geometry
    std::vector<MacroGeo> geo(nm);
    double hmin = INFINITY;
    for (int M = 0; M < nm; ++M) {
        MacroGeo& G = geo[M];
        std::memset(&G, 0, sizeof G);
        const double* p0 = vert + (size_t)mv[M * nvm] * d;
        double B[9] = {0}, Bi[9] = {0}, scale = 0;
        for (int i = 0; i < d; ++i) G.v0[i] = p0[i];
        for (int a = 0; a < d; ++a) {
            const double* pa = vert + (size_t)mv[M * nvm + a + 1] * d;
            for (int i = 0; i < d; ++i) {
                B[i * d + a] = pa[i] - p0[i];
                scale = std::max(scale, std::fabs(B[i * d + a]));
            }
        }
        const double det = invert(d, B, Bi);
        if (!(std::fabs(det) > 1e-12 * std::pow(scale, d)))
            return fail(c, MMOC_E_MESH, "macro %d is degenerate (det %.3g)", M, det);
        // shortest micro edge: the Kuhn lattice directions g_a = b_a - b_{a-1}
        // (b_0 = 0, b_a the macro edge v_a - v0) and their sums over
        // consecutive axes of some axis order, i.e. over every non-empty axis
        // subset at level >= 1; at level 0 the micro element is the macro
        {
            double g[3][3] = {};
            for (int a = 0; a < d; ++a)
                for (int i = 0; i < d; ++i) g[a][i] = B[i * d + a] - (a > 0 ? B[i * d + a - 1] : 0.0);
            for (int mask = 1; mask < (1 << d); ++mask) {
                bool contiguous = true;  // axes a..b without a gap: an edge of the macro itself
                int lo = -1, hi = -1;
                for (int a = 0; a < d; ++a)
                    if (mask & (1 << a)) {
                        if (lo < 0) lo = a;
                        hi = a;
                    }
                for (int a = lo; a <= hi; ++a) contiguous &= (mask >> a) & 1;
                if (c->level == 0 && !contiguous) continue;
                double v[3] = {};
                for (int a = 0; a < d; ++a)
                    if (mask & (1 << a))
                        for (int i = 0; i < d; ++i) v[i] += g[a][i];
                double len = 0.0;
                for (int i = 0; i < d; ++i) len += v[i] * v[i];
                hmin = std::min(hmin, std::sqrt(len) / c->n);
            }
        }
        for (int r = 0; r < d; ++r)
            for (int q = 0; q < d; ++q) {
                G.B[r * 3 + q] = B[r * d + q];
                G.binv[r * 3 + q] = Bi[r * d + q];
                G.binvf[r * 3 + q] = (float)Bi[r * d + q];
            }
        if (blend == MMOC_BLEND_SHELL_RADIAL) {
            // plane (2D: line) through the tips of the macro's d unit
            // directions: n' with n'.d_k = 1 for each direction d_k
            double dirs[3][3] = {};
            int nd = 0;
            for (int a = 0; a < nvm; ++a) {
                const double* p = vert + (size_t)mv[M * nvm + a] * d;
                double r2 = 0.0;
                for (int i = 0; i < d; ++i) r2 += p[i] * p[i];
                const double r = std::sqrt(r2);
                if (!(r > 0)) return fail(c, MMOC_E_MESH, "blended mesh has a vertex at the origin");
                double q[3] = {};
                for (int i = 0; i < d; ++i) q[i] = p[i] / r;
                bool dup = false;
                for (int b = 0; b < nd; ++b)
                    dup |= std::fabs(q[0] - dirs[b][0]) + std::fabs(q[1] - dirs[b][1]) + std::fabs(q[2] - dirs[b][2]) < 1e-9;
                if (!dup) {
                    if (nd == d) return fail(c, MMOC_E_MESH, "macro %d spans more than %d radial directions", M, d);
                    std::memcpy(dirs[nd++], q, sizeof q);
                }
            }
            if (nd != d) return fail(c, MMOC_E_MESH, "macro %d spans fewer than %d radial directions", M, d);
            double D[9], Di[9];
            for (int r = 0; r < d; ++r)
                for (int q = 0; q < d; ++q) D[r * d + q] = dirs[r][q];  // rows: directions
            const double dd = invert(d, D, Di);
            if (!(std::fabs(dd) > 1e-14)) return fail(c, MMOC_E_MESH, "macro %d has a flat column", M);
            double np[3] = {}, len2 = 0.0;
            for (int r = 0; r < d; ++r) {
                for (int q = 0; q < d; ++q) np[r] += Di[r * d + q];  // D n' = 1
                len2 += np[r] * np[r];
            }
            const double len = std::sqrt(len2);
            for (int r = 0; r < d; ++r) G.pn[r] = np[r] / len;
            G.pc = 1.0 / len;
        }
    }

    // --- faces: neighbours, manifoldness, conforming vertex order
    struct Face {
        std::array<int32_t, 3> key;
        int M, k;
    };
    std::vector<Face> faces;
    faces.reserve((size_t)nm * nvm);
    for (int M = 0; M < nm; ++M)
        for (int k = 0; k < nvm; ++k) {
            Face f{{-1, -1, -1}, M, k};
            int q = 0;
            for (int a = 0; a < nvm; ++a)
                if (a != k) f.key[q++] = mv[M * nvm + a];
            std::sort(f.key.begin(), f.key.begin() + d);
            faces.push_back(f);
        }
    std::sort(faces.begin(), faces.end(), [](const Face& a, const Face& b) {
        return a.key != b.key ? a.key < b.key : a.M < b.M;
    });
    for (int M = 0; M < nm; ++M)
        for (int k = 0; k < nvm; ++k) geo[M].nbr[k] = -1;
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j].key == faces[i].key) ++j;
        if (j - i > 2) return fail(c, MMOC_E_MESH, "face shared by %zu macros", j - i);
        if (j - i == 2) {
            const Face &a = faces[i], &b = faces[i + 1];
            // the face's vertices in local order must be the same sequence in both macros
            std::vector<int32_t> sa, sb;
            for (int q = 0; q < nvm; ++q) {
                if (q != a.k) sa.push_back(mv[a.M * nvm + q]);
                if (q != b.k) sb.push_back(mv[b.M * nvm + q]);
            }
            if (sa != sb)
                return fail(c, MMOC_E_MESH, "macros %d and %d order their shared face differently (non-conforming refinement)",
                            a.M, b.M);
            geo[a.M].nbr[a.k] = b.M;
            geo[b.M].nbr[b.k] = a.M;
        }
        i = j;
    }

    // --- owner of every sub-simplex, per macro and vertex subset
    const int nmask = 1 << nvm;
    std::map<std::array<int32_t, 4>, int> sub_owner;
    auto key_of = [&](int M, int mask) {
        std::array<int32_t, 4> k{{INT32_MAX, INT32_MAX, INT32_MAX, INT32_MAX}};
        int q = 0;
        for (int a = 0; a < nvm; ++a)
            if (mask >> a & 1) k[q++] = mv[M * nvm + a];
        std::sort(k.begin(), k.begin() + q);
        return k;
    };
    for (int M = 0; M < nm; ++M)
        for (int mask = 1; mask < nmask; ++mask) sub_owner.emplace(key_of(M, mask), M);  // first = lowest M
    std::vector<int32_t> mask_owner((size_t)nm * nmask);
    for (int M = 0; M < nm; ++M)
        for (int mask = 1; mask < nmask; ++mask) mask_owner[(size_t)M * nmask + mask] = sub_owner[key_of(M, mask)];

    // --- unique numbering and block slot map
    const int m = c->m;
    std::vector<int32_t> slot_uid((size_t)nm * npm);
    std::vector<uint64_t> owned;
    owned.reserve((size_t)nm * npm);
    std::vector<int32_t> own_slot;  // the slot where each DoF is owned (keep_chat)
    const bool keep = c->opt.keep_chat != 0;
    int64_t N = 0;
    for (int M = 0; M < nm; ++M) {
        int64_t idx = 0;
        for (int I = 0; I <= m; ++I)
            for (int J = 0; J <= I; ++J)
                for (int K = 0; K <= (d == 3 ? J : 0); ++K, ++idx) {
                    int w[4];
                    if (d == 2) {
                        w[0] = m - I; w[1] = I - J; w[2] = J; w[3] = 0;
                    } else {
                        w[0] = m - I; w[1] = I - J; w[2] = J - K; w[3] = K;
                    }
                    int mask = 0;
                    for (int a = 0; a < nvm; ++a)
                        if (w[a]) mask |= 1 << a;
                    const int Mo = mask_owner[(size_t)M * nmask + mask];
                    int32_t u;
                    if (Mo == M) {
                        u = (int32_t)N++;
                        owned.push_back(mmoc::pack_owned((uint32_t)M, (uint32_t)I, (uint32_t)J, (uint32_t)K));
                        if (keep) own_slot.push_back((int32_t)((int64_t)M * npm + idx));
                    } else {
                        // weights in the owner's local vertex order
                        int wo[4] = {0, 0, 0, 0};
                        for (int a = 0; a < nvm; ++a) {
                            if (!w[a]) continue;
                            const int g = mv[M * nvm + a];
                            for (int b = 0; b < nvm; ++b)
                                if (mv[Mo * nvm + b] == g) wo[b] = w[a];
                        }
                        int64_t io;
                        if (d == 2) io = lattice_index(2, wo[1] + wo[2], wo[2], 0);
                        else io = lattice_index(3, wo[1] + wo[2] + wo[3], wo[2] + wo[3], wo[3]);
                        u = slot_uid[(size_t)Mo * npm + io];
                    }
                    slot_uid[(size_t)M * npm + idx] = u;
                }
    }

    // --- upload
    c->nm = nm;
    c->hmin = hmin;
    c->npm = npm;
    c->nslots = (int64_t)nm * npm;
    c->N = N;
    c->blend = blend;
    mmoc_status st;
    if ((st = dev_alloc(c, &c->geo_d, nm, "geometry")) != MMOC_OK) return st;
    if ((st = dev_alloc(c, &c->owned_d, (size_t)N, "particle table")) != MMOC_OK) return st;
    if ((st = dev_alloc(c, &c->slot_uid_d, (size_t)c->nslots, "slot map")) != MMOC_OK) return st;
    const bool f32 = c->prec != MMOC_FP64;
    const size_t elem = f32 ? sizeof(float) : sizeof(double);
    if ((st = alloc_velocity_levels(c, c->lev_cap)) != MMOC_OK) return st;
    if ((st = alloc_clear(c, &c->cs_d, (size_t)c->nslots * elem, "scalar array")) != MMOC_OK) return st;
    std::vector<int32_t> dup;
    if (keep) {
        // the interface slots, each with the slot of its DoF's owner
        for (int64_t t = 0; t < c->nslots; ++t) {
            const int32_t o = own_slot[(size_t)slot_uid[(size_t)t]];
            if (o != (int32_t)t) {
                dup.push_back(o);
                dup.push_back((int32_t)t);
            }
        }
        c->ndup = (int64_t)dup.size() / 2;
        if ((st = alloc_clear(c, &c->cs_next, (size_t)c->nslots * elem, "next scalar array")) != MMOC_OK) return st;
        if (c->ndup > 0 && (st = dev_alloc(c, &c->dup_d, dup.size(), "interface slot list")) != MMOC_OK) return st;
    }
    c->chat_ready = false;
    HIPCHK(c, hipMemcpyAsync(c->geo_d, geo.data(), sizeof(MacroGeo) * nm, hipMemcpyHostToDevice, c->stream), "upload geometry");
    HIPCHK(c, hipMemcpyAsync(c->owned_d, owned.data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice, c->stream), "upload particles");
    HIPCHK(c, hipMemcpyAsync(c->slot_uid_d, slot_uid.data(), sizeof(int32_t) * c->nslots, hipMemcpyHostToDevice, c->stream),
           "upload slot map");
    if (!dup.empty())
        HIPCHK(c, hipMemcpyAsync(c->dup_d, dup.data(), sizeof(int32_t) * dup.size(), hipMemcpyHostToDevice, c->stream),
               "upload interface slot list");
    HIPCHK(c, hipStreamSynchronize(c->stream), "mesh upload");
    c->geo_h = std::move(geo);
    c->mesh_ok = true;
    return MMOC_OK;
}

mmoc_status mmoc_num_dofs(const mmoc_ctx* c, int64_t* n_unique, int64_t* n_block)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return MMOC_E_STATE;
    if (n_unique) *n_unique = c->N;
    if (n_block) *n_block = c->nslots;
    return MMOC_OK;
}

mmoc_status mmoc_dof_coords(mmoc_ctx* c, double* xyz)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    mmoc_status st = check_dev(c, xyz, sizeof(double) * c->dim * c->N, 8, "xyz_dev");
    if (st != MMOC_OK) return st;
    HIPCHK(c, mmoc::launch_dof_coords(c->dim, c->blend, c->geo_d, c->owned_d, c->N, c->m, xyz, c->stream), "dof_coords");
    return MMOC_OK;
}

// the record elements of velocity level `level` (ring slot) for components
// 0..dim-1 of u, appended to d from entry `first`
static void velocity_dst(mmoc_ctx* c, int level, const double* u, mmoc::ScatterDst& d, int first)
{
    const int L = phys_level(c, level);
    const size_t elem = c->prec == MMOC_FP64 ? sizeof(double) : sizeof(float);
    void* va = static_cast<char*>(c->va_all) + (size_t)L * c->va_lstride * elem;
    void* vb = c->vb_all ? static_cast<char*>(c->vb_all) + (size_t)L * c->vb_lstride * elem : nullptr;
    for (int i = 0; i < c->dim; ++i) d.src[first + i] = u + (size_t)i * c->N;
    if (c->dim == 3 && c->prec == MMOC_FP64) {
        d.dst[first] = d.dst[first + 1] = va;
        d.dst[first + 2] = vb;
        d.stride[first] = d.stride[first + 1] = 2;
        d.stride[first + 2] = c->zs;
        d.off[first] = 0;
        d.off[first + 1] = 1;
        d.off[first + 2] = 0;
    } else {
        const int na = c->dim == 3 ? 3 : 2;
        for (int i = 0; i < c->dim; ++i) {
            d.dst[first + i] = va;
            d.stride[first + i] = na;
            d.off[first + i] = i;
        }
    }
}

static mmoc_status check_velocity_level(mmoc_ctx* c, int level, const double* u)
{
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (level < 0 || level >= c->lev_cap)
        return fail(c, MMOC_E_ARG, "level must be in [0, %d] (the velocity levels held)", c->lev_cap - 1);
    if (c->stationary && level != 0) return fail(c, MMOC_E_STATE, "stationary velocity: only level 0 is used");
    return check_dev(c, u, sizeof(double) * c->dim * c->N, 8, "u_dev");
}

mmoc_status mmoc_set_velocity(mmoc_ctx* c, int level, const double* u)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = check_velocity_level(c, level, u);
    if (st != MMOC_OK) return st;
    mmoc::ScatterDst d{};
    velocity_dst(c, level, u, d, 0);
    HIPCHK(c, mmoc::launch_scatter(c->dim, c->slot_uid_d, c->nslots, c->N, d, c->prec != MMOC_FP64, c->stream),
           "set_velocity");
    c->vel_set[level] = true;
    return MMOC_OK;
}

mmoc_status mmoc_set_fields(mmoc_ctx* c, int level, const double* u, const double* cs)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = check_velocity_level(c, level, u);
    if (st != MMOC_OK) return st;
    if ((st = check_dev(c, cs, sizeof(double) * c->N, 8, "c_dev")) != MMOC_OK) return st;
    mmoc::ScatterDst d{};
    velocity_dst(c, level, u, d, 0);
    d.src[c->dim] = cs;
    d.dst[c->dim] = c->cs_d;
    d.stride[c->dim] = 1;
    d.off[c->dim] = 0;
    HIPCHK(c, mmoc::launch_scatter(c->dim + 1, c->slot_uid_d, c->nslots, c->N, d, c->prec != MMOC_FP64, c->stream),
           "set_fields");
    c->vel_set[level] = true;
    c->scalar_set = true;
    return MMOC_OK;
}

mmoc_status mmoc_set_stationary(mmoc_ctx* c, int on)
{
    if (!c) return MMOC_E_ARG;
    c->stationary = on != 0;
    if (c->stationary)
        for (int l = 1; l < c->lev_cap; ++l) c->vel_set[l] = 0;
    return MMOC_OK;
}

mmoc_status mmoc_swap_velocity_levels(mmoc_ctx* c)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (c->stationary) return fail(c, MMOC_E_STATE, "stationary velocity has one level");
    if (!c->vel_set[1]) return fail(c, MMOC_E_STATE, "velocity level 1 is not set");
    // the ring turns by one: logical level l takes the data of level l + 1,
    // and the last level (the oldest data) must be set again
    c->rot = (c->rot + 1) % c->lev_cap;
    for (int l = 0; l + 1 < c->lev_cap; ++l) c->vel_set[l] = c->vel_set[l + 1];
    c->vel_set[c->lev_cap - 1] = 0;
    return MMOC_OK;
}

mmoc_status mmoc_set_scalar(mmoc_ctx* c, const double* cs)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    mmoc_status st = check_dev(c, cs, sizeof(double) * c->N, 8, "c_dev");
    if (st != MMOC_OK) return st;
    mmoc::ScatterDst d{};
    d.src[0] = cs;
    d.dst[0] = c->cs_d;
    d.stride[0] = 1;
    d.off[0] = 0;
    HIPCHK(c, mmoc::launch_scatter(1, c->slot_uid_d, c->nslots, c->N, d, c->prec != MMOC_FP64, c->stream),
           "set_scalar");
    c->scalar_set = true;
    return MMOC_OK;
}

mmoc_status mmoc_use_last_chat(mmoc_ctx* c)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (!c->opt.keep_chat) return fail(c, MMOC_E_STATE, "options.keep_chat is off");
    if (!c->chat_ready) return fail(c, MMOC_E_STATE, "no trace call has written chat since the last use");
    std::swap(c->cs_d, c->cs_next);
    c->chat_ready = false;
    c->scalar_set = true;
    return MMOC_OK;
}

}  // extern "C"

// Shared by the plain and the surrogate step: launches the RK4 tracer on n
// particles whose unique ids are order[0..n) (all particles: the lane order).
mmoc_status mmoc_launch_trace(mmoc_ctx* c, double dt, int substeps, void* c_hat, double* X, const int32_t* order,
                              int64_t n, const unsigned long long* n_dev, int first, int n_int, const TraceExtra* ex)
{
    const hipStream_t stream = ex && ex->stream ? ex->stream : c->stream;
    auto fill = [&](auto& a) {
        a.geo = c->geo_d;
        a.owned = c->owned_d;
        a.order = order;
        a.n_dev = n_dev;
        a.n = n;
        a.xstride = c->N;
        a.nm = c->nm;
        a.npm = (int)c->npm;
        a.nlev = c->stationary ? 1 : 2;
        a.level_n = c->n;
        a.ord = c->opt.order;
        a.lat_m = c->m;
        a.substeps = substeps;
        a.max_hops = c->opt.max_hops;
        a.dt = dt;
        a.eps_in = c->opt.eps_in;
        a.eps32_macro = c->opt.eps32_macro;
        a.eps32_micro = c->opt.eps32_micro;
        a.elem_cache = c->opt.elem_cache;
        a.X = X;
        a.stats = c->stats_d;
        a.rk = c->rk;
        a.lsa = c->va_lstride;
        a.lsb = c->vb_lstride;
        a.zs = c->zs;
        a.lev_cap = c->lev_cap;
        a.rot = c->rot;
        a.first = first;
        a.n_int = n_int;
        a.checked = ex ? ex->checked : nullptr;
        a.xcheck = ex ? ex->xcheck : nullptr;
        a.tol_half = ex ? ex->tol_half : 0.0;
    };
    // keep_chat: a call that writes chat for every particle also writes the
    // next step's block-layout scalar (the trace kernel at each DoF's own
    // slot, then the interface slots from their owners)
    void* c_next = (c->opt.keep_chat && c_hat && !order && !n_dev && n == c->N) ? c->cs_next : nullptr;
    if (c->prec != MMOC_FP64) {
        mmoc::TraceArgs<float> a{};
        fill(a);
        a.va = (const float*)c->va_all;
        a.vb = (const float*)c->vb_all;
        a.cs = (const float*)c->cs_d;
        a.c_hat = (float*)c_hat;
        a.c_next = (float*)c_next;
        if (c->prec == MMOC_FP32_MIXED)
            HIPCHK(c, mmoc::launch_trace_fp32(c->dim, c->blend, a, stream), "trace (fp32 mixed)");
        else
            HIPCHK(c, mmoc::launch_trace_fp32_fields(c->dim, c->blend, a, stream), "trace (fp32 fields)");
    } else {
        mmoc::TraceArgs<double> a{};
        fill(a);
        a.va = (const double*)c->va_all;
        a.vb = (const double*)c->vb_all;
        a.cs = (const double*)c->cs_d;
        a.c_hat = (double*)c_hat;
        a.c_next = (double*)c_next;
        HIPCHK(c, mmoc::launch_trace_fp64(c->dim, c->blend, a, stream), "trace (fp64)");
    }
    if (c_next) {
        HIPCHK(c, mmoc::launch_dup_fill(c_next, c->prec != MMOC_FP64, c->dup_d, c->ndup, stream), "next scalar");
        c->chat_ready = true;
    }
    return MMOC_OK;
}

mmoc_status mmoc_check_step_args(mmoc_ctx* c, double dt, int substeps, void* c_hat, double* X)
{
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (!c->vel_set[0]) return fail(c, MMOC_E_STATE, "velocity level 0 is not set");
    if (!c->stationary && !c->vel_set[1]) return fail(c, MMOC_E_STATE, "velocity level 1 is not set (or set stationary)");
    if (!c->scalar_set) return fail(c, MMOC_E_STATE, "scalar is not set");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, MMOC_E_ARG, "dt must be positive and finite");
    if (substeps < 1 || substeps > (1 << 20)) return fail(c, MMOC_E_ARG, "substeps must be in [1, 2^20]");
    const size_t es = c->prec == MMOC_FP64 ? sizeof(double) : sizeof(float);
    mmoc_status st = check_dev(c, c_hat, es * c->N, es, "c_hat_dev");
    if (st != MMOC_OK) return st;
    if (X && (st = check_dev(c, X, sizeof(double) * c->dim * c->N, 8, "X_dev")) != MMOC_OK) return st;
    return MMOC_OK;
}

extern "C" {

mmoc_status mmoc_trace_step(mmoc_ctx* c, double dt, int substeps, void* c_hat, double* X)
{
    if (!c) return MMOC_E_ARG;
    mmoc_status st = mmoc_check_step_args(c, dt, substeps, c_hat, X);
    if (st != MMOC_OK) return st;
    return mmoc_launch_trace(c, dt, substeps, c_hat, X, nullptr, c->N);
}

mmoc_status mmoc_set_level_count(mmoc_ctx* c, int levels)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (levels < 2 || levels > 65536) return fail(c, MMOC_E_ARG, "levels must be in [2, 65536]");
    if (levels == c->lev_cap) return MMOC_OK;
    return alloc_velocity_levels(c, levels);
}

mmoc_status mmoc_trace_span(mmoc_ctx* c, int first, int n_int, double dt, int substeps, void* c_hat, double* X)
{
    if (!c) return MMOC_E_ARG;
    if (!c->mesh_ok) return fail(c, MMOC_E_STATE, "no mesh uploaded");
    if (n_int < 1) return fail(c, MMOC_E_ARG, "n_int must be at least 1");
    if (c->stationary) {
        if (first != 0) return fail(c, MMOC_E_ARG, "a stationary velocity has level 0 only");
        if (!c->vel_set[0]) return fail(c, MMOC_E_STATE, "velocity level 0 is not set");
    } else {
        if (first < 0 || first + n_int >= c->lev_cap)
            return fail(c, MMOC_E_ARG, "levels %d..%d are not all held (%d levels)", first, first + n_int, c->lev_cap);
        for (int l = first; l <= first + n_int; ++l)
            if (!c->vel_set[l]) return fail(c, MMOC_E_STATE, "velocity level %d is not set", l);
    }
    if (!c->scalar_set) return fail(c, MMOC_E_STATE, "scalar is not set");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, MMOC_E_ARG, "dt must be positive and finite");
    if (substeps < 1 || (int64_t)substeps * n_int > (1 << 20))
        return fail(c, MMOC_E_ARG, "substeps * n_int must be in [1, 2^20]");
    const size_t es = c->prec == MMOC_FP64 ? sizeof(double) : sizeof(float);
    mmoc_status st = check_dev(c, c_hat, es * c->N, es, "c_hat_dev");
    if (st != MMOC_OK) return st;
    if (X && (st = check_dev(c, X, sizeof(double) * c->dim * c->N, 8, "X_dev")) != MMOC_OK) return st;
    // a stationary field: one level, the whole span is one longer trace
    if (c->stationary) return mmoc_launch_trace(c, dt * n_int, substeps * n_int, c_hat, X, nullptr, c->N);
    return mmoc_launch_trace(c, dt, substeps, c_hat, X, nullptr, c->N, nullptr, first, n_int);
}

mmoc_status mmoc_get_stats(mmoc_ctx* c, mmoc_stats* out)
{
    if (!c || !out) return MMOC_E_ARG;
    unsigned long long w[mmoc::ST_COUNT * mmoc::kStatSpread];
    HIPCHK(c, hipMemcpyAsync(w, c->stats_d, sizeof w, hipMemcpyDeviceToHost, c->stream), "read stats");
    HIPCHK(c, hipStreamSynchronize(c->stream), "read stats");
    // each counter is spread over kStatSpread words: sum them (max for the residual bits)
    unsigned long long h[mmoc::ST_COUNT] = {};
    for (int k = 0; k < mmoc::ST_COUNT; ++k)
        for (int j = 0; j < mmoc::kStatSpread; ++j) {
            const unsigned long long v = w[k * mmoc::kStatSpread + j];
            if (k == mmoc::ST_MAXRES_BITS) h[k] = v > h[k] ? v : h[k];
            else h[k] += v;
        }
    out->n_particles = (int64_t)h[mmoc::ST_PARTICLES];
    out->n_outside = (int64_t)h[mmoc::ST_OUTSIDE];
    out->n_multi_hop = (int64_t)h[mmoc::ST_MULTIHOP];
    out->n_bruteforce = (int64_t)h[mmoc::ST_BRUTE];
    out->n_tieband = (int64_t)h[mmoc::ST_TIEBAND];
    out->n_nan = (int64_t)h[mmoc::ST_NAN];
    out->n_checked = (int64_t)h[mmoc::ST_CHECKED];
    out->n_fallback = (int64_t)h[mmoc::ST_FALLBACK];
    double r;
    std::memcpy(&r, &h[mmoc::ST_MAXRES_BITS], sizeof r);
    out->max_check_residual = r;
    out->n_cache_lookups = (int64_t)h[mmoc::ST_CACHE_LOOKUPS];
    out->n_cache_hits = (int64_t)h[mmoc::ST_CACHE_HITS];
    return MMOC_OK;
}

mmoc_status mmoc_reset_stats(mmoc_ctx* c)
{
    if (!c) return MMOC_E_ARG;
    HIPCHK(c, hipMemsetAsync(c->stats_d, 0, sizeof(unsigned long long) * mmoc::ST_COUNT * mmoc::kStatSpread, c->stream),
           "reset stats");
    return MMOC_OK;
}

const char* mmoc_last_error(const mmoc_ctx* c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

void mmoc_destroy(mmoc_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"

namespace {
void free_all(mmoc_ctx* c)
{
    mmoc_mlp_free_state(c);
    mmoc_fe_free_state(c);
    (void)hipFree(c->geo_d);
    (void)hipFree(c->owned_d);
    (void)hipFree(c->slot_uid_d);
    (void)hipFree(c->va_all);
    (void)hipFree(c->vb_all);
    c->va_all = c->vb_all = nullptr;
    (void)hipFree(c->cs_d);
    (void)hipFree(c->cs_next);
    (void)hipFree(c->dup_d);
    (void)hipFree(c->stats_d);
    (void)hipFree(c->red_d);
    c->red_d = nullptr;
    c->red_cap = 0;
    c->geo_d = nullptr;
    c->owned_d = nullptr;
    c->slot_uid_d = nullptr;
    c->cs_d = nullptr;
    c->cs_next = nullptr;
    c->dup_d = nullptr;
    c->ndup = 0;
    c->chat_ready = false;
    c->stats_d = nullptr;
}
}  // namespace

// Context lifecycle: mesh copies, the 4x4 block pattern of the condensed
// system, the element-to-block map and every device workspace.
//
// The condensed system couples the (v, p) unknowns of two nodes exactly when
// they share an element (Section 5: the condensed blocks are assembled from
// element-level 4-node contributions), so the pattern is the node graph of
// the mesh plus the diagonal, stored as block-CSR with 4x4 blocks.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include <map>

#include "vms_internal.h"

namespace {
thread_local std::string g_last_error;
}

namespace vms {

int set_error(vms_ctx* ctx, int code, const std::string& msg) {
    g_last_error = msg;
    if (ctx) ctx->err = msg;
    return code;
}

int check_hip(vms_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return VMS_OK;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return set_error(ctx, e == hipErrorOutOfMemory ? VMS_ENOMEM : VMS_EHIP, buf);
}

}  // namespace vms

using namespace vms;

extern "C" const char* vms_last_error(const vms_ctx* ctx) {
    if (ctx && !ctx->err.empty()) return ctx->err.c_str();
    return g_last_error.c_str();
}

namespace vms {

static constexpr int kProfPool = 4096;

static int prof_flush(vms_ctx* c) {
    for (int i = 0; i < c->prof_used; ++i) {
        hipEvent_t e0 = c->prof_ev[2 * i], e1 = c->prof_ev[2 * i + 1];
        if (hipEventSynchronize(e1) != hipSuccess) return VMS_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return VMS_EHIP;
        const int ph = c->prof_phase[i];
        if (ph < 0) continue;           // voided: the launch did no work
        c->prof_ms[ph] += ms;
        c->prof_acc_bytes[ph] += c->prof_bytes[i];
        c->prof_count[ph] += 1;
    }
    c->prof_used = 0;
    ++c->prof_gen;
    return VMS_OK;
}

int prof_begin(vms_ctx* c, int phase, double bytes, hipStream_t s) {
    if (!c->prof_force && c->prof_seen[phase]++ % c->prof_every != 0) return -1;
    if (c->prof_used == kProfPool && prof_flush(c) != VMS_OK) return -1;
    const int slot = c->prof_used++;
    c->prof_phase[slot] = phase;
    c->prof_bytes[slot] = bytes;
    (void)hipEventRecord(c->prof_ev[2 * slot], s);
    return slot;
}

void prof_end(vms_ctx* c, int slot, hipStream_t s) { (void)hipEventRecord(c->prof_ev[2 * slot + 1], s); }

void prof_void(vms_ctx* c, int slot, int64_t gen) {
    if (slot >= 0 && gen == c->prof_gen && slot < c->prof_used) c->prof_phase[slot] = -1;
}

}  // namespace vms

extern "C" int vms_profile(vms_ctx* c, uint32_t phase_mask, int32_t every) {
    if (!c) return set_error(nullptr, VMS_EINVAL, "vms_profile: NULL ctx");
    if (phase_mask & ~VMS_PROFILE_ALL) return set_error(c, VMS_EINVAL, "vms_profile: unknown phase bit");
    if (every < 1) return set_error(c, VMS_EINVAL, "vms_profile: every must be >= 1");
    if (c->prof_ev.empty() && phase_mask) {
        c->prof_ev.resize(2 * kProfPool);
        for (auto& e : c->prof_ev)
            // timing-only events: no system-scope fence (cache write-back) around the timed launches
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess)
                return set_error(c, VMS_EHIP, "vms_profile: hipEventCreate");
        c->prof_phase.resize(kProfPool);
        c->prof_bytes.resize(kProfPool);
    }
    if (c->prof_used && prof_flush(c) != VMS_OK) return set_error(c, VMS_EHIP, "vms_profile: event sync");
    for (int i = 0; i < VMS_NPHASES; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_acc_bytes[i] = 0.0;
        c->prof_count[i] = 0;
    }
    c->prof_mask = phase_mask;
    c->prof_every = every;
    for (int i = 0; i < VMS_NPHASES; ++i) c->prof_seen[i] = 0;
    c->prof_cycles = 0;
    return VMS_OK;
}

extern "C" int vms_profile_read(vms_ctx* c, double* ms, int64_t* launches, double* alg_bytes) {
    if (!c) return set_error(nullptr, VMS_EINVAL, "vms_profile_read: NULL ctx");
    if (c->prof_used && prof_flush(c) != VMS_OK) return set_error(c, VMS_EHIP, "vms_profile_read: event sync");
    for (int i = 0; i < VMS_NPHASES; ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (launches) launches[i] = c->prof_count[i];
        if (alg_bytes) alg_bytes[i] = c->prof_acc_bytes[i];
    }
    return VMS_OK;
}

static void free_all(vms_ctx* c) {
    if (c->full) {
        free_all(c->full);
        delete c->full;
        c->full = nullptr;
    }
    void* ptrs[] = {c->full_cc, c->full_epos, c->zfull, c->xyz4, c->tets, c->dmask, c->dlist, c->rowptr, c->colidx, c->diagpos,
                    c->tpos, c->tile_meta, c->tile_nodes, c->items, c->bmask, c->tile_part, c->A, c->rhs, c->du, c->rnorm, c->flags,
                    c->V, c->w, c->z, c->d, c->r, c->Minv, c->AP, c->Az, c->x64, c->r64, c->gs, c->red,
                    c->feats, c->hid, c->pblk, c->gblk, c->gdel, c->tvec, c->wgrad, c->fscal, c->dr_p,
                    c->V64, c->w64, c->z64};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto e : c->prof_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->progress_host) (void)hipHostFree(c->progress_host);
    if (c->dr_pinned) (void)hipHostFree(c->dr_pinned);
    if (c->cycle_exec) (void)hipGraphExecDestroy(c->cycle_exec);
    for (hipGraphExec_t& e : c->dr_exec)
        if (e) (void)hipGraphExecDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
}

extern "C" int vms_destroy(vms_ctx* ctx) {
    if (!ctx) return VMS_OK;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_all(ctx);
    (void)hipSetDevice(dev);
    delete ctx;
    return VMS_OK;
}

template <class P>
static int dev_alloc(vms_ctx* c, P** p, size_t bytes, const char* what) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes ? bytes : 16);
    return check_hip(c, e, what);
}

#define TRY(x)                     \
    do {                           \
        int rc__ = (x);            \
        if (rc__ != VMS_OK) {      \
            free_all(c);           \
            delete c;              \
            return rc__;           \
        }                          \
    } while (0)

// The uncondensed Newton system as a 4x4 block-CSR system over nn + ne block rows: node rows
// hold their node-node blocks (the condensed pattern's columns, in the same order) followed by
// one block per adjacent element; element rows hold the blocks of their four nodes (sorted)
// followed by the diagonal block.  The solver-only child context gets the pattern, the masks
// (the unused fourth dof of an element row is masked like a Dirichlet dof) and the Krylov
// workspaces; the parent keeps the positions of the element contributions.
static int create_full_system(vms_ctx* c, const std::vector<int32_t>& tets, const std::vector<int32_t>& n2e_ptr,
                              const std::vector<int32_t>& n2e, const std::vector<int32_t>& rowptr,
                              const std::vector<int32_t>& colidx, const std::vector<int32_t>& diagpos,
                              const std::vector<uint8_t>& dmask) {
    const int64_t nn = c->n_nodes, ne = c->n_elems, nr = nn + ne;
    const int64_t nbf = c->nb + 9 * ne;
    if (nbf >= (int64_t)INT32_MAX / 16 || 4 * nr >= (int64_t)INT32_MAX)
        return set_error(c, VMS_EINVAL, "vms_create: uncondensed system exceeds int32 indexing");
    std::vector<int32_t> fptr(nr + 1), fcol(nbf), fdiag(nr), fcc(c->nb), fepos(9 * ne);
    std::vector<uint8_t> fmask(nr);
    int64_t k = 0;
    for (int64_t i = 0; i < nn; ++i) {
        fptr[i] = (int32_t)k;
        for (int32_t b = rowptr[i]; b < rowptr[i + 1]; ++b) {
            fcc[b] = (int32_t)k;
            fcol[k++] = colidx[b];
        }
        fdiag[i] = fptr[i] + (diagpos[i] - rowptr[i]);
        for (int32_t q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) fcol[k++] = (int32_t)(nn + n2e[q]);
        fmask[i] = dmask[i];
    }
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t row = nn + e;
        fptr[row] = (int32_t)k;
        int32_t sorted[4] = {tets[4 * e], tets[4 * e + 1], tets[4 * e + 2], tets[4 * e + 3]};
        std::sort(sorted, sorted + 4);
        for (int a = 0; a < 4; ++a) fcol[k + a] = sorted[a];
        for (int b = 0; b < 4; ++b)
            fepos[9 * e + 4 + b] = (int32_t)(k + (std::find(sorted, sorted + 4, tets[4 * e + b]) - sorted));
        fcol[k + 4] = (int32_t)row;
        fdiag[row] = (int32_t)(k + 4);
        fepos[9 * e + 8] = (int32_t)(k + 4);
        k += 5;
        fmask[row] = 8u;
    }
    fptr[nr] = (int32_t)k;
    if (k != nbf) return set_error(c, VMS_EINVAL, "vms_create: uncondensed pattern size mismatch");
    // (node a, element e): the position of e in node a's element list
    for (int64_t i = 0; i < nn; ++i) {
        const int32_t first = fptr[i] + (rowptr[i + 1] - rowptr[i]);
        for (int32_t q = n2e_ptr[i]; q < n2e_ptr[i + 1]; ++q) {
            const int32_t e = n2e[q];
            for (int a = 0; a < 4; ++a)
                if (tets[4 * (int64_t)e + a] == i) fepos[9 * (int64_t)e + a] = first + (q - n2e_ptr[i]);
        }
    }

    vms_ctx* f = new vms_ctx();
    c->full = f;
    f->device = c->device;
    f->prec = c->prec;
    f->max_restart = c->max_restart;
    f->n_pressure_pins = c->n_pressure_pins;
    f->n_nodes = (int32_t)nr;
    f->full_nodes = c->n_nodes;
    f->n_elems = 0;
    f->nb = nbf;
    const size_t es = elt_size(c);
    const size_t N = 4 * (size_t)nr;
    int rc;
#define FTRY(x)                  \
    do {                         \
        if ((rc = (x)) != VMS_OK) { \
            if (!f->err.empty()) c->err = f->err; \
            return rc;           \
        }                        \
    } while (0)
    FTRY(dev_alloc(c, &c->full_cc, c->nb * sizeof(int32_t), "alloc full map"));
    FTRY(dev_alloc(c, &c->full_epos, 9 * ne * sizeof(int32_t), "alloc full map"));
    FTRY(dev_alloc(f, &f->rowptr, (nr + 1) * sizeof(int32_t), "alloc full rowptr"));
    FTRY(dev_alloc(f, &f->colidx, nbf * sizeof(int32_t), "alloc full colidx"));
    FTRY(dev_alloc(f, &f->diagpos, nr * sizeof(int32_t), "alloc full diagpos"));
    FTRY(dev_alloc(f, &f->dmask, nr, "alloc full dmask"));
    FTRY(dev_alloc(f, &f->A, nbf * 16 * es, "alloc full A"));
    FTRY(dev_alloc(f, &f->rhs, N * sizeof(double), "alloc full rhs"));
    FTRY(dev_alloc(f, &f->du, N * sizeof(double), "alloc full du"));
    FTRY(dev_alloc(f, &f->rnorm, 8 * sizeof(double), "alloc full rnorm"));
    FTRY(dev_alloc(f, &f->flags, 8 * sizeof(int32_t), "alloc full flags"));
    FTRY(dev_alloc(f, &f->V, (size_t)(f->max_restart + 1) * N * es, "alloc full Krylov basis"));
    FTRY(dev_alloc(f, &f->w, N * es, "alloc full w"));
    FTRY(dev_alloc(f, &f->z, N * es, "alloc full z"));
    FTRY(dev_alloc(f, &f->d, N * es, "alloc full d"));
    FTRY(dev_alloc(f, &f->r, N * es, "alloc full r"));
    FTRY(dev_alloc(f, &f->Minv, nr * 16 * es, "alloc full Minv"));
    FTRY(dev_alloc(f, &f->AP, nbf * 16 * es, "alloc full A P"));
    FTRY(dev_alloc(f, &f->Az, N * es, "alloc full A z"));
    FTRY(dev_alloc(f, &f->zfull, N * sizeof(double), "alloc full coarse vector"));
    FTRY(dev_alloc(f, &f->x64, N * sizeof(double), "alloc full x64"));
    FTRY(dev_alloc(f, &f->r64, N * sizeof(double), "alloc full r64"));
    FTRY(dev_alloc(f, &f->tvec, 3 * N * sizeof(float), "alloc full tvec"));
    FTRY(dev_alloc(f, &f->gs, sizeof(GmresState), "alloc full gmres state"));
    FTRY(dev_alloc(f, &f->red, sizeof(RedScratch), "alloc full reduction scratch"));
    FTRY(check_hip(f, hipHostMalloc(reinterpret_cast<void**>(&f->progress_host), 128,
                                    hipHostMallocMapped | hipHostMallocCoherent), "alloc progress word"));
    FTRY(check_hip(f, hipHostGetDevicePointer(reinterpret_cast<void**>(&f->progress_dev), f->progress_host, 0),
                   "map progress word"));
    for (int i = 0; i < 8; ++i) f->progress_host[i] = 0;      // progress word, norm tags
    f->scal_host = reinterpret_cast<double*>(f->progress_host + 8);
    f->scal_dev = reinterpret_cast<double*>(f->progress_dev + 8);
    for (int i = 0; i < 8; ++i) f->scal_host[i] = 0.0;
    FTRY(check_hip(c, hipMemcpy(c->full_cc, fcc.data(), c->nb * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    FTRY(check_hip(c, hipMemcpy(c->full_epos, fepos.data(), 9 * ne * sizeof(int32_t), hipMemcpyHostToDevice),
                   "upload"));
    FTRY(check_hip(f, hipMemcpy(f->rowptr, fptr.data(), (nr + 1) * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    FTRY(check_hip(f, hipMemcpy(f->colidx, fcol.data(), nbf * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    FTRY(check_hip(f, hipMemcpy(f->diagpos, fdiag.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    FTRY(check_hip(f, hipMemcpy(f->dmask, fmask.data(), nr, hipMemcpyHostToDevice), "upload"));
    FTRY(check_hip(f, hipMemset(f->red, 0, sizeof(RedScratch)), "clear"));
    FTRY(check_hip(f, hipMemset(f->gs, 0, sizeof(GmresState)), "clear"));
    FTRY(check_hip(f, hipMemset(f->flags, 0, 8 * sizeof(int32_t)), "clear"));
    FTRY(check_hip(f, hipMemcpy(&f->gs->progress, &f->progress_dev, sizeof(uint64_t*), hipMemcpyHostToDevice),
                   "upload"));
#undef FTRY
    return VMS_OK;
}

extern "C" int vms_create(const vms_mesh_desc* mesh, const vms_create_opts* opts,
                          hipStream_t stream, vms_ctx** out) {
    if (!out) return set_error(nullptr, VMS_EINVAL, "vms_create: out is NULL");
    *out = nullptr;
    if (!mesh || !mesh->xyz || !mesh->tets || mesh->n_nodes <= 0 || mesh->n_elems <= 0)
        return set_error(nullptr, VMS_EINVAL, "vms_create: empty or NULL mesh");
    if (mesh->n_dirichlet < 0 || (mesh->n_dirichlet > 0 && !mesh->dirichlet_dofs))
        return set_error(nullptr, VMS_EINVAL, "vms_create: bad Dirichlet list");
    if ((int64_t)mesh->n_nodes * 4 >= (int64_t)INT32_MAX)
        return set_error(nullptr, VMS_EINVAL, "vms_create: too many nodes for int32 dofs");

    vms_ctx* c = new vms_ctx();
    c->n_nodes = mesh->n_nodes;
    c->n_elems = mesh->n_elems;
    c->n_dir = mesh->n_dirichlet;
    c->prec = opts ? opts->precision : VMS_FP64;
    c->max_restart = (opts && opts->max_restart > 0) ? opts->max_restart : 50;
    if (c->prec != VMS_FP64 && c->prec != VMS_MIXED) {
        delete c;
        return set_error(nullptr, VMS_EINVAL, "vms_create: unknown precision");
    }
    if (c->max_restart > kMaxRestart) {
        delete c;
        return set_error(nullptr, VMS_EINVAL, "vms_create: max_restart above 128");
    }
    TRY(check_hip(c, hipGetDevice(&c->device), "hipGetDevice"));

    const int64_t nn = c->n_nodes, ne = c->n_elems;
    std::vector<double> xyz(3 * nn);
    std::vector<int32_t> tets(4 * ne);
    std::vector<int32_t> dl(c->n_dir);
    TRY(check_hip(c, hipMemcpyAsync(xyz.data(), mesh->xyz, 3 * nn * sizeof(double),
                                    hipMemcpyDeviceToHost, stream), "copy xyz"));
    TRY(check_hip(c, hipMemcpyAsync(tets.data(), mesh->tets, 4 * ne * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, stream), "copy tets"));
    if (c->n_dir)
        TRY(check_hip(c, hipMemcpyAsync(dl.data(), mesh->dirichlet_dofs, c->n_dir * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, stream), "copy dirichlet"));
    TRY(check_hip(c, hipStreamSynchronize(stream), "sync"));

    // validate connectivity and orientation
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t* t = &tets[4 * e];
        for (int a = 0; a < 4; ++a)
            if (t[a] < 0 || t[a] >= nn) {
                free_all(c);
                delete c;
                return set_error(nullptr, VMS_EINVAL, "vms_create: node index out of range in element " +
                                                          std::to_string(e));
            }
        const double* x0 = &xyz[3 * t[0]];
        double J[3][3];
        for (int k = 0; k < 3; ++k)
            for (int i = 0; i < 3; ++i) J[i][k] = xyz[3 * t[k + 1] + i] - x0[i];
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(det > 0.0)) {
            free_all(c);
            delete c;
            return set_error(nullptr, VMS_EDEGENERATE,
                             "vms_create: element " + std::to_string(e) + " has det J <= 0");
        }
    }
    std::vector<uint8_t> dmask(nn, 0);
    for (int32_t d : dl) {
        if (d < 0 || d >= 4 * nn) {
            free_all(c);
            delete c;
            return set_error(nullptr, VMS_EINVAL, "vms_create: Dirichlet dof out of range");
        }
        dmask[d >> 2] |= (uint8_t)(1u << (d & 3));
    }
    for (int32_t i = 0; i < nn; ++i) c->n_pressure_pins += (dmask[i] >> 3) & 1;

    // node -> elements
    std::vector<int32_t> n2e_ptr(nn + 1, 0), n2e;
    for (int64_t i = 0; i < 4 * ne; ++i) n2e_ptr[tets[i] + 1]++;
    for (int64_t i = 0; i < nn; ++i) n2e_ptr[i + 1] += n2e_ptr[i];
    n2e.resize(n2e_ptr[nn]);
    {
        std::vector<int32_t> fill(n2e_ptr.begin(), n2e_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < 4; ++a) n2e[fill[tets[4 * e + a]]++] = (int32_t)e;
    }
    // rows of the block pattern: sorted unique neighbours (including self)
    std::vector<int32_t> rowptr(nn + 1, 0), colidx;
    colidx.reserve(16 * nn);
    std::vector<int32_t> scratch;
    for (int64_t i = 0; i < nn; ++i) {
        scratch.clear();
        for (int32_t k = n2e_ptr[i]; k < n2e_ptr[i + 1]; ++k) {
            const int32_t* t = &tets[4 * (int64_t)n2e[k]];
            scratch.insert(scratch.end(), t, t + 4);
        }
        if (scratch.empty()) scratch.push_back((int32_t)i);   // isolated node: diagonal only
        std::sort(scratch.begin(), scratch.end());
        scratch.erase(std::unique(scratch.begin(), scratch.end()), scratch.end());
        colidx.insert(colidx.end(), scratch.begin(), scratch.end());
        rowptr[i + 1] = (int32_t)colidx.size();
    }
    c->nb = (int64_t)colidx.size();
    if (c->nb >= (int64_t)INT32_MAX / 16) {
        free_all(c);
        delete c;
        return set_error(nullptr, VMS_EINVAL, "vms_create: block count exceeds int32 indexing");
    }
    auto find = [&](int32_t row, int32_t col) -> int32_t {
        const int32_t* b = colidx.data() + rowptr[row];
        const int32_t* e = colidx.data() + rowptr[row + 1];
        const int32_t* p = std::lower_bound(b, e, col);
        return (int32_t)(p - colidx.data());
    };
    std::vector<int32_t> diagpos(nn), tpos(c->nb);
    for (int64_t i = 0; i < nn; ++i) {
        diagpos[i] = find((int32_t)i, (int32_t)i);
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) tpos[k] = find(colidx[k], (int32_t)i);
    }

    struct Quad {
        int32_t e[4];
        int n;          // elements taken (the rest are zero-weight copies of e[0])
        int32_t j;      // neighbour shared by all four elements, or -1
    };
    // Assembly tiles: contiguous node ranges whose block rows fit the LDS budget and whose
    // elements touch at most kTileMaxNodes distinct nodes (their coordinates and state are staged
    // in LDS).  Local node numbering per tile: the owned nodes first, in order, then the other
    // vertices of the tile's elements in increasing global order.
    const size_t acc_size = c->prec == VMS_FP64 ? sizeof(double) : kMixedAccSize;
    const bool det = opts && opts->deterministic;
    c->tile_threads = det ? 64 : 256;
    // DPP quads in the FP32-block tiles (the FP64 kernel has no registers left for the quad
    // exchanges)
    const bool quads = c->prec == VMS_MIXED;
    int64_t max_blocks = det ? kTileBlocksDet : acc_size == sizeof(double) ? kTileBlocksFP64 : kTileBlocksFP32;
    if (det) {
        // a one-wavefront tile still holds the longest row of the pattern
        int64_t longest = 0;
        for (int64_t i = 0; i < nn; ++i) longest = std::max<int64_t>(longest, rowptr[i + 1] - rowptr[i]);
        max_blocks = std::max(max_blocks, longest);
    }
    std::vector<int32_t> tnode0{0}, tiptr{0}, tnptr{0}, tnodes;
    std::vector<uint4> items;
    items.reserve(4 * ne);
    size_t lds_max = 0, lds_max_tr = 0;
    {
        std::vector<int32_t> stamp(nn, -1), loc(nn, 0), cand, halo;
        int64_t r0 = 0;
        int32_t tile = 0;
        while (r0 < nn) {
            if (rowptr[r0 + 1] - rowptr[r0] > max_blocks) {
                free_all(c);
                delete c;
                return set_error(nullptr, VMS_EINVAL, "vms_create: node " + std::to_string(r0) +
                                                          " has more block neighbours than an assembly tile holds");
            }
            int64_t r1 = r0;
            int32_t ndist = 0;
            while (r1 < nn && r1 - r0 < kTileNodes && rowptr[r1 + 1] - rowptr[r0] <= max_blocks) {
                cand.clear();
                if (stamp[r1] != tile) cand.push_back((int32_t)r1);
                for (int32_t k = n2e_ptr[r1]; k < n2e_ptr[r1 + 1]; ++k)
                    for (int a = 0; a < 4; ++a) {
                        const int32_t v = tets[4 * (int64_t)n2e[k] + a];
                        if (stamp[v] != tile) cand.push_back(v);
                    }
                std::sort(cand.begin(), cand.end());
                cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
                if (ndist + (int64_t)cand.size() > kTileMaxNodes) break;
                for (int32_t v : cand) stamp[v] = tile;
                ndist += (int32_t)cand.size();
                ++r1;
            }
            if (r1 == r0) {
                free_all(c);
                delete c;
                return set_error(nullptr, VMS_EINVAL, "vms_create: the elements around node " + std::to_string(r0) +
                                                          " touch more nodes than an assembly tile stages");
            }
            halo.clear();
            for (int64_t i = r0; i < r1; ++i) {
                loc[i] = (int32_t)(i - r0);
                for (int32_t k = n2e_ptr[i]; k < n2e_ptr[i + 1]; ++k)
                    for (int a = 0; a < 4; ++a) {
                        const int32_t v = tets[4 * (int64_t)n2e[k] + a];
                        if (v < r0 || v >= r1) halo.push_back(v);
                    }
            }
            std::sort(halo.begin(), halo.end());
            halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
            for (size_t j = 0; j < halo.size(); ++j) loc[halo[j]] = (int32_t)(r1 - r0 + (int64_t)j);
            for (int64_t i = r0; i < r1; ++i) tnodes.push_back((int32_t)i);
            tnodes.insert(tnodes.end(), halo.begin(), halo.end());
            const int64_t ntn = (r1 - r0) + (int64_t)halo.size();
            // Mixed-precision tiles take their items in quads: four consecutive items (the four
            // lanes of a DPP quad) belong to one owned row, so the kernel reduce-scatters their
            // diagonal block and residual rows over the quad and each lane adds a quarter of
            // them.  A row's elements are grouped greedily by a shared edge (i, j) where four of
            // them still share one; such a quad puts j at local position 1 in all four items and
            // shares that block too.  A row's last quad is padded with zero-weight copies.  The
            // quads that share an edge come first, then the others, so that few wavefronts hold
            // both kinds; within each kind they go round-robin over the owned rows (the r-th
            // quad of every row, then the (r+1)-th), so that the quads of a wavefront mostly
            // add into different rows.
            // Without quads (quads == false) every quad holds one item: the items of the owned rows
            // go round-robin (the r-th element of every owned row, then the (r+1)-th, ...).
            std::vector<std::vector<Quad>> row_quads(r1 - r0);
            int32_t rounds = 0;
            for (int64_t i = r0; i < r1; ++i) {
                auto& qs = row_quads[i - r0];
                std::vector<int32_t> rem(n2e.begin() + n2e_ptr[i], n2e.begin() + n2e_ptr[i + 1]);
                while (!rem.empty()) {
                    Quad q{};
                    q.j = -1;
                    if (!quads) {
                        q.e[0] = rem.front();
                        q.n = 1;
                        rem.erase(rem.begin());
                        qs.push_back(q);
                        continue;
                    }
                    if (rem.size() >= 4) {
                        // the neighbour shared by the most remaining elements
                        std::map<int32_t, int> cnt;
                        for (int32_t e : rem)
                            for (int b = 0; b < 4; ++b) {
                                const int32_t v = tets[4 * (int64_t)e + b];
                                if (v != i) cnt[v]++;
                            }
                        int32_t best = -1;
                        int bc = 0;
                        for (auto& kv : cnt)
                            if (kv.second > bc) best = kv.first, bc = kv.second;
                        if (bc >= 4) q.j = best;
                    }
                    int taken = 0;
                    for (size_t k = 0; k < rem.size() && taken < 4;) {
                        const int32_t e = rem[k];
                        bool has = q.j < 0;
                        for (int b = 0; b < 4 && !has; ++b) has = tets[4 * (int64_t)e + b] == q.j;
                        if (has) {
                            q.e[taken++] = e;
                            rem.erase(rem.begin() + k);
                        } else {
                            ++k;
                        }
                    }
                    q.n = taken;
                    qs.push_back(q);
                }
                rounds = std::max(rounds, (int32_t)qs.size());
            }
            const int32_t b0 = rowptr[r0];
            for (int kind = 0; kind < 2; ++kind) {
                for (int32_t r = 0; r < rounds; ++r)
                    for (int64_t i = r0; i < r1; ++i) {
                        // kind 0: the r-th quad of row i that shares an edge; kind 1: the r-th other one
                        const auto& qs = row_quads[i - r0];
                        int32_t seen = -1;
                        const Quad* qp = nullptr;
                        for (const Quad& cand : qs)
                            if ((cand.j >= 0) == (kind == 0) && ++seen == r) {
                                qp = &cand;
                                break;
                            }
                        if (!qp) continue;
                        const Quad& q = *qp;
                        for (int m = 0; m < (quads ? 4 : 1); ++m) {
                            const bool dummy = m >= q.n;
                            const int32_t e = q.e[dummy ? 0 : m];
                            const int32_t* t = &tets[4 * (int64_t)e];
                            int a = 0;
                            while (t[a] != i) ++a;
                            // vertex order: the owned vertex a first, then j (when the quad shares it),
                            // then the others, as an even permutation of (0, 1, 2, 3)
                            int ord[4] = {a, a ^ 1, a ^ 2, a ^ 3};
                            if (q.j >= 0) {
                                int pj = 1;
                                while (t[ord[pj]] != q.j) ++pj;
                                if (pj != 1) {
                                    // rotate positions 1..3 (an even permutation) until j is at 1
                                    while (t[ord[1]] != q.j) {
                                        const int x = ord[1];
                                        ord[1] = ord[2];
                                        ord[2] = ord[3];
                                        ord[3] = x;
                                    }
                                }
                            }
                            uint32_t pslot[4], l = 0;
                            for (int b = 0; b < 4; ++b) {
                                pslot[b] = (uint32_t)(find((int32_t)i, t[ord[b]]) - b0);
                                l |= (uint32_t)loc[t[ord[b]]] << (8 * b);
                            }
                            // x: element (bit 31: zero-weight copy); y: local node numbers; z: slots
                            // 0, 1 (bit 15: the element's vertex 0, counted once in the norm); w:
                            // slots 2, 3 (bit 31: the quad shares slot 1)
                            items.push_back(make_uint4((uint32_t)e | (dummy ? 0x80000000u : 0u), l,
                                                       pslot[0] | ((a == 0 && !dummy) ? 0x8000u : 0u) | (pslot[1] << 16),
                                                       pslot[2] | (pslot[3] << 16) | (q.j >= 0 ? 0x80000000u : 0u)));
                        }
                    }
            }
            tnode0.push_back((int32_t)r1);
            tiptr.push_back((int32_t)items.size());
            tnptr.push_back((int32_t)tnodes.size());
            const size_t base = tile_lds_bytes(rowptr[r1] - rowptr[r0], r1 - r0, acc_size);
            lds_max = std::max(lds_max, base + (size_t)ntn * 64);
            lds_max_tr = std::max(lds_max_tr, base + (size_t)ntn * 96);
            r0 = r1;
            ++tile;
        }
    }
    c->n_tiles = (int32_t)(tnode0.size() - 1);
    c->tile_lds = lds_max;
    c->tile_lds_tr = lds_max_tr;

    std::vector<double> xyz4(4 * nn);
    for (int64_t i = 0; i < nn; ++i) {
        xyz4[4 * i + 0] = xyz[3 * i + 0];
        xyz4[4 * i + 1] = xyz[3 * i + 1];
        xyz4[4 * i + 2] = xyz[3 * i + 2];
        xyz4[4 * i + 3] = 0.0;
    }

    const size_t es = elt_size(c);
    const size_t N = 4 * (size_t)nn;
    TRY(dev_alloc(c, &c->xyz4, nn * sizeof(double4), "alloc xyz"));
    TRY(dev_alloc(c, &c->tets, ne * sizeof(int4), "alloc tets"));
    TRY(dev_alloc(c, &c->dmask, nn, "alloc dmask"));
    TRY(dev_alloc(c, &c->dlist, c->n_dir * sizeof(int32_t), "alloc dlist"));
    TRY(dev_alloc(c, &c->rowptr, (nn + 1) * sizeof(int32_t), "alloc rowptr"));
    TRY(dev_alloc(c, &c->colidx, c->nb * sizeof(int32_t), "alloc colidx"));
    TRY(dev_alloc(c, &c->diagpos, nn * sizeof(int32_t), "alloc diagpos"));
    TRY(dev_alloc(c, &c->tpos, c->nb * sizeof(int32_t), "alloc tpos"));
    TRY(dev_alloc(c, &c->tile_meta, 2 * (size_t)c->n_tiles * sizeof(int4), "alloc tiles"));
    TRY(dev_alloc(c, &c->tile_nodes, tnodes.size() * sizeof(int32_t), "alloc tile nodes"));
    TRY(dev_alloc(c, &c->items, items.size() * sizeof(uint4), "alloc tile items"));
    TRY(dev_alloc(c, &c->bmask, c->nb * sizeof(uint16_t), "alloc block masks"));
    TRY(dev_alloc(c, &c->tile_part, 2 * (size_t)c->n_tiles * sizeof(double), "alloc tile partials"));
    TRY(dev_alloc(c, &c->A, c->nb * 16 * es, "alloc A"));
    TRY(dev_alloc(c, &c->rhs, N * sizeof(double), "alloc rhs"));
    TRY(dev_alloc(c, &c->du, N * sizeof(double), "alloc du"));
    TRY(dev_alloc(c, &c->rnorm, 8 * sizeof(double), "alloc rnorm"));
    TRY(dev_alloc(c, &c->flags, 8 * sizeof(int32_t), "alloc flags"));
    TRY(dev_alloc(c, &c->V, (size_t)(c->max_restart + 1) * N * es, "alloc Krylov basis"));
    TRY(dev_alloc(c, &c->w, N * es, "alloc w"));
    TRY(dev_alloc(c, &c->z, N * es, "alloc z"));
    TRY(dev_alloc(c, &c->d, N * es, "alloc d"));
    TRY(dev_alloc(c, &c->r, N * es, "alloc r"));
    TRY(dev_alloc(c, &c->Minv, nn * 16 * es, "alloc Minv"));
    TRY(dev_alloc(c, &c->AP, c->nb * 16 * es, "alloc A P"));
    TRY(dev_alloc(c, &c->Az, N * es, "alloc A z"));
    TRY(dev_alloc(c, &c->x64, N * sizeof(double), "alloc x64"));
    TRY(dev_alloc(c, &c->r64, N * sizeof(double), "alloc r64"));
    TRY(dev_alloc(c, &c->gs, sizeof(GmresState), "alloc gmres state"));
    TRY(dev_alloc(c, &c->dr_p, sizeof(double) * kDrUpload, "alloc deflation upload"));
    TRY(check_hip(c, hipHostMalloc(&c->dr_pinned, kDrStagingBytes), "alloc deflation staging"));
    if (c->prec == VMS_MIXED && opts && opts->basis_fp64) {
        TRY(dev_alloc(c, &c->V64, (size_t)(c->max_restart + 1) * N * sizeof(double), "alloc FP64 Krylov basis"));
        TRY(dev_alloc(c, &c->w64, N * sizeof(double), "alloc FP64 w"));
        TRY(dev_alloc(c, &c->z64, N * sizeof(double), "alloc FP64 z"));
    }
    TRY(dev_alloc(c, &c->red, sizeof(RedScratch), "alloc reduction scratch"));
    TRY(dev_alloc(c, &c->feats, nn * VMS_PC_NIN * sizeof(float), "alloc feats"));
    TRY(dev_alloc(c, &c->hid, nn * VMS_PC_NHID * sizeof(float), "alloc hidden"));
    TRY(dev_alloc(c, &c->pblk, nn * 16 * sizeof(float), "alloc pblk"));
    TRY(dev_alloc(c, &c->gblk, nn * 16 * sizeof(float), "alloc gblk"));
    TRY(dev_alloc(c, &c->gdel, nn * 16 * sizeof(float), "alloc gdel"));
    TRY(dev_alloc(c, &c->tvec, 3 * N * sizeof(float), "alloc tvec"));
    TRY(dev_alloc(c, &c->wgrad, (size_t)kRedBlocks * VMS_PC_NWEIGHTS * sizeof(float), "alloc wgrad"));
    TRY(dev_alloc(c, &c->fscal, 8 * sizeof(float), "alloc fscal"));
    TRY(check_hip(c, hipHostMalloc(reinterpret_cast<void**>(&c->progress_host), 128,
                                   hipHostMallocMapped | hipHostMallocCoherent), "alloc progress word"));
    TRY(check_hip(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->progress_dev), c->progress_host, 0),
                  "map progress word"));
    for (int i = 0; i < 8; ++i) c->progress_host[i] = 0;      // progress word, norm tags
    c->scal_host = reinterpret_cast<double*>(c->progress_host + 8);
    c->scal_dev = reinterpret_cast<double*>(c->progress_dev + 8);
    for (int i = 0; i < 8; ++i) c->scal_host[i] = 0.0;
    TRY(check_hip(c, hipEventCreate(&c->ev0), "event"));
    TRY(check_hip(c, hipEventCreate(&c->ev1), "event"));

    std::vector<int4> t4(ne);
    for (int64_t e = 0; e < ne; ++e)
        t4[e] = make_int4(tets[4 * e], tets[4 * e + 1], tets[4 * e + 2], tets[4 * e + 3]);
    TRY(check_hip(c, hipMemcpy(c->xyz4, xyz4.data(), nn * sizeof(double4), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->tets, t4.data(), ne * sizeof(int4), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->dmask, dmask.data(), nn, hipMemcpyHostToDevice), "upload"));
    if (c->n_dir)
        TRY(check_hip(c, hipMemcpy(c->dlist, dl.data(), c->n_dir * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->rowptr, rowptr.data(), (nn + 1) * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->colidx, colidx.data(), c->nb * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->diagpos, diagpos.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->tpos, tpos.data(), c->nb * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    {
        std::vector<int4> meta(2 * (size_t)c->n_tiles);
        for (int32_t t = 0; t < c->n_tiles; ++t) {
            meta[2 * t] = make_int4(tnode0[t], tnode0[t + 1], rowptr[tnode0[t]], rowptr[tnode0[t + 1]] - rowptr[tnode0[t]]);
            meta[2 * t + 1] = make_int4(tiptr[t], tiptr[t + 1], tnptr[t], tnptr[t + 1] - tnptr[t]);
        }
        TRY(check_hip(c, hipMemcpy(c->tile_meta, meta.data(), meta.size() * sizeof(int4), hipMemcpyHostToDevice),
                      "upload"));
    }
    TRY(check_hip(c, hipMemcpy(c->tile_nodes, tnodes.data(), tnodes.size() * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemcpy(c->items, items.data(), items.size() * sizeof(uint4), hipMemcpyHostToDevice), "upload"));
    {
        std::vector<uint16_t> bm(c->nb);
        for (int64_t i = 0; i < nn; ++i)
            for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                bm[k] = (uint16_t)((dmask[colidx[k]] & 0xFu) | ((dmask[i] & 0xFu) << 4) | (colidx[k] == i ? 0x100u : 0u));
        TRY(check_hip(c, hipMemcpy(c->bmask, bm.data(), c->nb * sizeof(uint16_t), hipMemcpyHostToDevice), "upload"));
    }
    TRY(check_hip(c, tile_kernels_configure(c), "configure tile kernels"));
    TRY(check_hip(c, hipMemset(c->red, 0, sizeof(RedScratch)), "clear"));
    TRY(check_hip(c, hipMemset(c->gs, 0, sizeof(GmresState)), "clear"));
    TRY(check_hip(c, hipMemcpy(&c->gs->progress, &c->progress_dev, sizeof(uint64_t*), hipMemcpyHostToDevice),
                  "upload"));
    if (opts && opts->full_system)
        TRY(create_full_system(c, tets, n2e_ptr, n2e, rowptr, colidx, diagpos, dmask));
    TRY(check_hip(c, hipMemset(c->flags, 0, 8 * sizeof(int32_t)), "clear"));
    TRY(noalloc_scratch_init(c));
    TRY(check_hip(c, hipDeviceSynchronize(), "sync"));
    *out = c;
    return VMS_OK;
}

extern "C" int vms_set_linearization(vms_ctx* ctx, int kind) {
    if (!ctx) return set_error(nullptr, VMS_EINVAL, "vms_set_linearization: NULL ctx");
    if (kind != VMS_LIN_NEWTON && kind != VMS_LIN_PICARD)
        return set_error(ctx, VMS_EINVAL, "vms_set_linearization: unknown kind");
    ctx->linearization = kind;
    return VMS_OK;
}

extern "C" int vms_full_info(const vms_ctx* ctx, int64_t* nb, int32_t* n_rows, const int32_t** rowptr,
                             const int32_t** colidx) {
    if (!ctx) return set_error(nullptr, VMS_EINVAL, "vms_full_info: NULL ctx");
    if (!ctx->full) return set_error(const_cast<vms_ctx*>(ctx), VMS_EINVAL,
                                     "vms_full_info: context created without full_system");
    if (nb) *nb = ctx->full->nb;
    if (n_rows) *n_rows = ctx->full->n_nodes;
    if (rowptr) *rowptr = ctx->full->rowptr;
    if (colidx) *colidx = ctx->full->colidx;
    return VMS_OK;
}

extern "C" int vms_bsr_info(const vms_ctx* ctx, int64_t* nb, const int32_t** rowptr,
                            const int32_t** colidx, const int32_t** diagpos, int32_t* precision) {
    if (!ctx) return set_error(nullptr, VMS_EINVAL, "vms_bsr_info: NULL ctx");
    if (nb) *nb = ctx->nb;
    if (rowptr) *rowptr = ctx->rowptr;
    if (colidx) *colidx = ctx->colidx;
    if (diagpos) *diagpos = ctx->diagpos;
    if (precision) *precision = (int32_t)ctx->prec;
    return VMS_OK;
}

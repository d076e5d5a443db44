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

static void free_all(vms_ctx* c) {
    void* ptrs[] = {c->xyz4, c->tets, c->dmask, c->dlist, c->rowptr, c->colidx, c->diagpos,
                    c->tpos, c->epos, c->A, c->rhs, c->du, c->rglob, c->rnorm, c->flags,
                    c->V, c->w, c->z, c->d, c->r, c->Minv, c->x64, c->r64, c->gs, c->red,
                    c->feats, c->hid, c->pblk, c->gblk, c->tvec, c->wgrad, c->fscal};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
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
    std::vector<int32_t> diagpos(nn), tpos(c->nb), epos(16 * ne);
    for (int64_t i = 0; i < nn; ++i) {
        diagpos[i] = find((int32_t)i, (int32_t)i);
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) tpos[k] = find(colidx[k], (int32_t)i);
    }
    for (int64_t e = 0; e < ne; ++e)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                epos[(a * 4 + b) * ne + e] = find(tets[4 * e + a], tets[4 * e + b]);

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
    TRY(dev_alloc(c, &c->epos, 16 * ne * sizeof(int32_t), "alloc epos"));
    TRY(dev_alloc(c, &c->A, c->nb * 16 * es, "alloc A"));
    TRY(dev_alloc(c, &c->rhs, N * sizeof(double), "alloc rhs"));
    TRY(dev_alloc(c, &c->du, N * sizeof(double), "alloc du"));
    TRY(dev_alloc(c, &c->rglob, N * sizeof(double), "alloc rglob"));
    TRY(dev_alloc(c, &c->rnorm, 8 * sizeof(double), "alloc rnorm"));
    TRY(dev_alloc(c, &c->flags, 8 * sizeof(int32_t), "alloc flags"));
    TRY(dev_alloc(c, &c->V, (size_t)(c->max_restart + 1) * N * es, "alloc Krylov basis"));
    TRY(dev_alloc(c, &c->w, N * es, "alloc w"));
    TRY(dev_alloc(c, &c->z, N * es, "alloc z"));
    TRY(dev_alloc(c, &c->d, N * es, "alloc d"));
    TRY(dev_alloc(c, &c->r, N * es, "alloc r"));
    TRY(dev_alloc(c, &c->Minv, nn * 16 * es, "alloc Minv"));
    TRY(dev_alloc(c, &c->x64, N * sizeof(double), "alloc x64"));
    TRY(dev_alloc(c, &c->r64, N * sizeof(double), "alloc r64"));
    TRY(dev_alloc(c, &c->gs, sizeof(GmresState), "alloc gmres state"));
    TRY(dev_alloc(c, &c->red, sizeof(RedScratch), "alloc reduction scratch"));
    TRY(dev_alloc(c, &c->feats, nn * VMS_PC_NIN * sizeof(float), "alloc feats"));
    TRY(dev_alloc(c, &c->hid, nn * VMS_PC_NHID * sizeof(float), "alloc hidden"));
    TRY(dev_alloc(c, &c->pblk, nn * 16 * sizeof(float), "alloc pblk"));
    TRY(dev_alloc(c, &c->gblk, nn * 16 * sizeof(float), "alloc gblk"));
    TRY(dev_alloc(c, &c->tvec, 3 * N * sizeof(float), "alloc tvec"));
    TRY(dev_alloc(c, &c->wgrad, (size_t)kRedBlocks * VMS_PC_NWEIGHTS * sizeof(float), "alloc wgrad"));
    TRY(dev_alloc(c, &c->fscal, 8 * sizeof(float), "alloc fscal"));
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
    TRY(check_hip(c, hipMemcpy(c->epos, epos.data(), 16 * ne * sizeof(int32_t), hipMemcpyHostToDevice), "upload"));
    TRY(check_hip(c, hipMemset(c->red, 0, sizeof(RedScratch)), "clear"));
    TRY(check_hip(c, hipMemset(c->gs, 0, sizeof(GmresState)), "clear"));
    TRY(check_hip(c, hipMemset(c->flags, 0, 8 * sizeof(int32_t)), "clear"));
    TRY(check_hip(c, hipDeviceSynchronize(), "sync"));
    *out = c;
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

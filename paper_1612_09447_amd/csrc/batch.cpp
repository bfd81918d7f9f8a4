// Batched form: many independent instances packed into one context (see
// eqs_set_instances), plus the convenience calls that build such a context
// from separately described instances and step it.
#include <algorithm>
#include <cstring>

#include "eqs_internal.h"

struct eqs_batch {
    eqs_ctx* packed = nullptr;
    int32_t n = 0;
    std::vector<int64_t> node_off;
    double* d_x = nullptr;  // packed potentials (owned by the packed context's allocations)
    std::vector<int64_t> iters;
    std::vector<double> relres;
};

extern "C" {

int eqs_batch_create(eqs_batch** out, int32_t n, eqs_ctx* const* ctxs, int device, void* hip_stream,
                     const eqs_amg_params* p) {
    if (!out || !ctxs || n < 1) {
        eqs::set_error("eqs_batch_create: NULL argument or n < 1");
        return EQS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    std::vector<double> xyz;
    std::vector<int32_t> tets, tet_mat, dnodes, ddrive;
    std::vector<eqs_material> mats;
    std::vector<eqs_drive> drives;
    std::vector<int64_t> noff{0}, toff{0};
    for (int32_t i = 0; i < n; ++i) {
        const eqs_ctx* c = ctxs[i];
        if (!c || !(c->have_mesh && c->have_mat && c->have_dir)) {
            eqs::set_error("eqs_batch_create: instance " + std::to_string(i) + " lacks mesh, materials or Dirichlet data");
            return EQS_ERR_STATE;
        }
        if (c->npe != 4) {
            eqs::set_error("eqs_batch_create: batches hold first-order (4-node) meshes");
            return EQS_ERR_INVALID_ARG;
        }
        const int32_t nbase = (int32_t)noff.back();
        const int32_t mbase = (int32_t)mats.size();
        const int32_t dbase = (int32_t)drives.size();
        xyz.insert(xyz.end(), c->xyz.begin(), c->xyz.end());
        for (int32_t v : c->tets) tets.push_back(v + nbase);
        for (int32_t m : c->tet_mat) tet_mat.push_back(m + mbase);
        mats.insert(mats.end(), c->mats.begin(), c->mats.end());
        for (size_t k = 0; k < c->dir_nodes.size(); ++k) {
            dnodes.push_back(c->dir_nodes[k] + nbase);
            ddrive.push_back(c->dir_drive[k] + dbase);
        }
        drives.insert(drives.end(), c->drives.begin(), c->drives.end());
        noff.push_back(noff.back() + c->n_nodes);
        toff.push_back(toff.back() + c->n_tets);
    }
    eqs_batch* b = new eqs_batch();
    b->n = n;
    b->node_off = noff;
    b->iters.assign(n, 0);
    b->relres.assign(n, 0.0);
    int rc;
    if ((rc = eqs_create(&b->packed, device, hip_stream)) != EQS_OK ||
        (rc = eqs_set_mesh(b->packed, noff.back(), xyz.data(), toff.back(), tets.data())) != EQS_OK ||
        (rc = eqs_set_instances(b->packed, n, noff.data(), toff.data())) != EQS_OK ||
        (rc = eqs_set_materials(b->packed, (int32_t)mats.size(), mats.data(), tet_mat.data())) != EQS_OK ||
        (rc = eqs_set_dirichlet(b->packed, (int64_t)dnodes.size(), dnodes.data(), ddrive.data(), (int32_t)drives.size(),
                                drives.data())) != EQS_OK ||
        (rc = eqs_build_preconditioner(b->packed, p)) != EQS_OK) {
        std::string msg = eqs_last_error();
        eqs_destroy(b->packed);
        delete b;
        eqs::set_error("eqs_batch_create: " + msg);
        return rc;
    }
    try {
        b->d_x = (double*)eqs::dev_alloc(b->packed, sizeof(double) * (size_t)noff.back());
    } catch (const eqs::Error& e) {
        eqs_destroy(b->packed);
        delete b;
        eqs::set_error(e.msg);
        return e.code;
    }
    *out = b;
    return EQS_OK;
}

int eqs_batch_set_graph_iters(eqs_batch* b, int32_t iters) {
    if (!b) {
        eqs::set_error("eqs_batch_set_graph_iters: NULL batch");
        return EQS_ERR_INVALID_ARG;
    }
    return eqs_set_graph_iters(b->packed, iters);
}

int eqs_batch_destroy(eqs_batch* b) {
    if (!b) return EQS_OK;
    eqs_destroy(b->packed);
    delete b;
    return EQS_OK;
}

int eqs_batch_rkc_steps(eqs_batch* b, int32_t nsteps, double t0, double dt, int32_t s, double* const* x_dev,
                        double rtol, int32_t maxit, eqs_step_stats* st) {
    if (!b || !x_dev || nsteps < 0) {
        eqs::set_error("eqs_batch_rkc_steps: NULL argument or nsteps < 0");
        return EQS_ERR_INVALID_ARG;
    }
    eqs_ctx* c = b->packed;
    try {
        EQS_HIP(hipSetDevice(c->device));
        for (int32_t i = 0; i < b->n; ++i) {
            if (!x_dev[i]) throw eqs::Error{EQS_ERR_INVALID_ARG, "eqs_batch_rkc_steps: NULL x_dev entry"};
            EQS_HIP(hipMemcpyAsync(b->d_x + b->node_off[i], x_dev[i],
                                   sizeof(double) * (size_t)(b->node_off[i + 1] - b->node_off[i]),
                                   hipMemcpyDeviceToDevice, c->stream));
        }
    } catch (const eqs::Error& e) {
        eqs::set_error(e.msg);
        return e.code;
    }
    std::fill(b->iters.begin(), b->iters.end(), 0);
    std::fill(b->relres.begin(), b->relres.end(), 0.0);
    std::vector<int64_t> it(b->n);
    std::vector<double> rr(b->n);
    int rc_all = EQS_OK;
    for (int32_t k = 0; k < nsteps; ++k) {
        const int rc = eqs_rkc_step(c, t0 + k * dt, dt, s, b->d_x, rtol, maxit, st);
        if (rc != EQS_OK && rc != EQS_ERR_NOT_CONVERGED) return rc;
        if (rc == EQS_ERR_NOT_CONVERGED) rc_all = rc;
        eqs_instance_stats(c, b->n, it.data(), rr.data());
        for (int32_t i = 0; i < b->n; ++i) {
            b->iters[i] += it[i];
            b->relres[i] = std::max(b->relres[i], rr[i]);
        }
    }
    try {
        for (int32_t i = 0; i < b->n; ++i)
            EQS_HIP(hipMemcpyAsync(x_dev[i], b->d_x + b->node_off[i],
                                   sizeof(double) * (size_t)(b->node_off[i + 1] - b->node_off[i]),
                                   hipMemcpyDeviceToDevice, c->stream));
        EQS_HIP(hipStreamSynchronize(c->stream));
    } catch (const eqs::Error& e) {
        eqs::set_error(e.msg);
        return e.code;
    }
    return rc_all;
}

int eqs_batch_instance_stats(const eqs_batch* b, int64_t* iters, double* relres) {
    if (!b) {
        eqs::set_error("eqs_batch_instance_stats: NULL argument");
        return EQS_ERR_INVALID_ARG;
    }
    for (int32_t i = 0; i < b->n; ++i) {
        if (iters) iters[i] = b->iters[i];
        if (relres) relres[i] = b->relres[i];
    }
    return EQS_OK;
}

}  // extern "C"

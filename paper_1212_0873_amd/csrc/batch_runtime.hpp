// batch_runtime.hpp -- host side of the batched solver and of the schedule
// autotuner (included by pcdm.hip: one translation unit owns every kernel).
#pragma once

#include "batch_kernels.hpp"

struct pcdm_batch {
    int count = 0;
    int dtype = PCDM_F32;
    size_t vb = 4, tbytes = 4;
    int nblk_max = 2048;
    std::vector<BatchInst> hdesc;
    std::vector<int32_t> hactive;
    std::vector<int64_t> omega, stored, k_host;
    std::vector<double> beta, lambda, atb_inf;
    uint64_t seed = 0;

    char *seg = nullptr;
    int64_t *pc_all = nullptr;
    double *x = nullptr, *r64 = nullptr, *b = nullptr, *acc = nullptr;  // acc: 4 + 4 per problem
    // incremental ||A_j^T r_j||_inf: r of the last evaluation, per-column
    // upper bounds and norms (rounded up), per problem [M_old, max norm, -, valid]
    double *rold = nullptr, *ist = nullptr;
    float *ubc = nullptr, *nrmc = nullptr;
    int incremental = 1;
    std::vector<int64_t> inc_evals, cands;  // per problem: evaluations that moved bounds, last candidates
    std::vector<char> inc_state;
    void *r = nullptr, *delta_slot = nullptr;
    int32_t *id_slot = nullptr, *active = nullptr;
    BatchInst *desc = nullptr;
    int32_t *step_tiles = nullptr;
    int64_t n_step_tiles = 0;
    int64_t n_col_tiles = 0, n_row_tiles = 0;  // over all problems
    uint64_t *nz_part = nullptr;
    BatchList list{nullptr, nullptr, nullptr, nullptr};  // problems of the current refresh / objective pass

    // objective: problems evaluated by the next call (device copy of hsel),
    // and the last values of each problem with the step count they hold for
    // (a problem that has not stepped since keeps them)
    int32_t *sel = nullptr;
    std::vector<int32_t> hsel;
    std::vector<double> cF, cG;
    std::vector<int64_t> ck;
    std::vector<char> cvalid;

    int lanes = 4, chunks = 1;
    int64_t graph_len = 32;  // steps per captured graph; 0 = no graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t graph_captured_len = 0;
};

namespace {

void batch_drop_graph(pcdm_batch *B)
{
    if (B->exec)
        (void)hipGraphExecDestroy(B->exec);
    if (B->graph)
        (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_captured_len = 0;
}

void batch_free(pcdm_batch *B)
{
    if (!B)
        return;
    batch_drop_graph(B);
    void *bufs[] = {B->seg, B->pc_all, B->x, B->r64, B->b, B->acc, B->rold, B->ist, B->ubc, B->nrmc,
                    B->r, B->delta_slot, B->id_slot, B->active,
                    B->desc, B->step_tiles, B->nz_part, B->sel, B->list.n, B->list.ids, B->list.colp,
                    B->list.rowp};
    for (void *q : bufs)
        if (q)
            (void)hipFree(q);
    if (B->cap_stream)
        (void)hipStreamDestroy(B->cap_stream);
    delete B;
}

template <typename V> struct BatchOps {
    using T = typename ValT<V>::T;

    template <int G, int C> static void launch_step(pcdm_batch *B, hipStream_t s)
    {
        const int gs = grid_for(B->n_step_tiles * 64, kBlock, B->nblk_max);
        hipLaunchKernelGGL((k_batch_gather<V, G, C>), dim3(gs), dim3(kBlock), 0, s, B->seg,
                           (const BatchInst *)B->desc, (const int32_t *)B->active, (const int32_t *)B->step_tiles,
                           B->n_step_tiles, (const T *)B->r, B->x, B->id_slot, (T *)B->delta_slot, B->nz_part);
        hipLaunchKernelGGL((k_batch_scatter<V, G>), dim3(gs), dim3(kBlock), 0, s, (const char *)B->seg, B->desc,
                           (const int32_t *)B->active, B->count, (const int32_t *)B->step_tiles, B->n_step_tiles,
                           (T *)B->r, (const int32_t *)B->id_slot, (const T *)B->delta_slot, B->list);
        refresh(B, s);  // the scatter listed the due problems
        hipLaunchKernelGGL((k_batch_narrow<T>), dim3(grid_for(B->n_row_tiles * 64, kBlock, B->nblk_max)),
                           dim3(kBlock), 0, s, (const BatchInst *)B->desc, B->list, (const double *)B->r64,
                           (T *)B->r);
    }

    static int step_once(pcdm_batch *B, hipStream_t s)
    {
        switch (B->lanes * 16 + B->chunks) {
        case 1 * 16 + 1: launch_step<1, 1>(B, s); break;
        case 1 * 16 + 2: launch_step<1, 2>(B, s); break;
        case 1 * 16 + 4: launch_step<1, 4>(B, s); break;
        case 2 * 16 + 1: launch_step<2, 1>(B, s); break;
        case 2 * 16 + 2: launch_step<2, 2>(B, s); break;
        case 2 * 16 + 4: launch_step<2, 4>(B, s); break;
        case 4 * 16 + 1: launch_step<4, 1>(B, s); break;
        case 4 * 16 + 2: launch_step<4, 2>(B, s); break;
        case 8 * 16 + 1: launch_step<8, 1>(B, s); break;
        case 8 * 16 + 2: launch_step<8, 2>(B, s); break;
        case 16 * 16 + 1: launch_step<16, 1>(B, s); break;
        case 32 * 16 + 1: launch_step<32, 1>(B, s); break;
        case 64 * 16 + 1: launch_step<64, 1>(B, s); break;
        default: return fail(PCDM_EINVAL, "unsupported (lanes_per_column, chunks_per_lane) pair");
        }
        return PCDM_OK;
    }

    // B->list = the problems due after this step, or (sel given) those with
    // sel[j] != 0.
    static void list(pcdm_batch *B, hipStream_t s, const int32_t *sel)
    {
        hipLaunchKernelGGL(k_batch_list, dim3(1), dim3(kBlock), 0, s, (const BatchInst *)B->desc,
                           (const int32_t *)B->active, B->count, sel, B->list);
    }

    // r64 = A x - b for the listed problems.
    static void refresh(pcdm_batch *B, hipStream_t s)
    {
        hipLaunchKernelGGL(k_batch_neg_b, dim3(grid_for(B->n_row_tiles * 64, kBlock, B->nblk_max)), dim3(kBlock), 0,
                           s, (const BatchInst *)B->desc, B->list, (const double *)B->b, B->r64);
        hipLaunchKernelGGL((k_batch_refresh_cols<V, 8>), dim3(grid_for(B->n_col_tiles * 64, kBlock, B->nblk_max)),
                           dim3(kBlock), 0, s, (const char *)B->seg, (const BatchInst *)B->desc, B->list,
                           (const double *)B->x, B->r64);
    }

    // acc[4j..4j+3] for the problems with B->sel[j] != 0 (others zero).
    static void objective(pcdm_batch *B, hipStream_t s)
    {
        list(B, s, B->sel);
        refresh(B, s);
        double *dacc = B->acc + 4 * (int64_t)B->count;
        hipLaunchKernelGGL((k_fill<double>), dim3(1), dim3(kBlock), 0, s, B->acc, 0.0, (int64_t)8 * B->count);
        hipLaunchKernelGGL(k_batch_row_sums, dim3(grid_for(B->n_row_tiles * 64, kBlock, B->nblk_max)),
                           dim3(kBlock), 0, s, (const BatchInst *)B->desc, B->list, (const double *)B->b,
                           (const double *)B->r64, B->acc, B->rold, dacc);
        hipLaunchKernelGGL((k_batch_col_obj<V, 8>), dim3(grid_for(B->n_col_tiles * 64, kBlock, B->nblk_max)),
                           dim3(kBlock), 0, s, (const char *)B->seg, (const BatchInst *)B->desc, B->list,
                           (const double *)B->x, (const double *)B->r64, B->acc, B->ubc, (const float *)B->nrmc,
                           (const double *)B->ist, dacc, B->incremental);
        hipLaunchKernelGGL(k_batch_keep_max, dim3(1), dim3(kBlock), 0, s, B->list, (const double *)B->acc,
                           B->ist);
    }

    // nrmc of problem j's columns (>= ||a_i||_1, float32 rounded up) and
    // ist[4j+1] = their maximum.
    static void col_norms(pcdm_batch *B, int j, double *part, hipStream_t s)
    {
        const BatchInst &d = B->hdesc[j];
        const double dmax = d.lay.fixed_dpad ? (double)d.lay.fixed_dpad : (double)d.m;
        const int g = grid_for(d.n, kBlock, B->nblk_max);
        hipLaunchKernelGGL((k_col_norms<V, 8>), dim3(g), dim3(kBlock), 0, s, (const char *)B->seg + d.rec_base, d.lay,
                           d.n, inc_l1_factor(dmax), B->nrmc + d.col_base, part);
        hipLaunchKernelGGL(k_final, dim3(1), dim3(kBlock), 0, s, (const double *)part, g, 1, 1, B->ist + 4 * j + 1);
    }

    static void narrow_all(pcdm_batch *B, hipStream_t s)
    {
        // at k = 0 every active problem is due
        list(B, s, nullptr);
        hipLaunchKernelGGL((k_batch_narrow<T>), dim3(grid_for(B->n_row_tiles * 64, kBlock, B->nblk_max)),
                           dim3(kBlock), 0, s, (const BatchInst *)B->desc, B->list, (const double *)B->r64,
                           (T *)B->r);
    }

    static void pack(pcdm_batch *B, const int64_t *col_ptr, const int32_t *rows, const void *vals, int j,
                     int32_t *hist, Ctrl *ctrl, hipStream_t s)
    {
        const BatchInst &d = B->hdesc[j];
        hipLaunchKernelGGL((k_pack<V>), dim3(grid_for(d.n, kBlock, B->nblk_max)), dim3(kBlock), 0, s, col_ptr, rows,
                           (const V *)vals, d.lay, d.n, d.m, B->seg + d.rec_base, hist, ctrl);
    }
};

template <typename F> int batch_dispatch(int dtype, F &&f)
{
    switch (dtype) {
    case PCDM_F32: return f(BatchOps<float>());
    case PCDM_BF16: return f(BatchOps<bf16s>());
    case PCDM_F64: return f(BatchOps<double>());
    default: return fail(PCDM_EINVAL, "unknown dtype");
    }
}

int batch_step_direct(pcdm_batch *B, hipStream_t s)
{
    return batch_dispatch(B->dtype, [&](auto ops) { return decltype(ops)::step_once(B, s); });
}

int batch_capture(pcdm_batch *B)
{
    batch_drop_graph(B);
    if (!B->cap_stream)
        HIP_TRY(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal));
    int st = PCDM_OK;
    for (int64_t q = 0; q < B->graph_len && st == PCDM_OK; ++q)
        st = batch_step_direct(B, B->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->cap_stream, &g);
    if (st != PCDM_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return hip_fail(e, "hipStreamEndCapture");
    B->graph = g;
    HIP_TRY(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    B->graph_captured_len = B->graph_len;
    return PCDM_OK;
}

bool valid_instance(const pcdm_csc *A, double lambda, int64_t tau, std::string &why)
{
    if (!A) {
        why = "NULL matrix";
        return false;
    }
    if (A->m < 1 || A->n < 1 || A->n > INT32_MAX - 1 || A->m > INT32_MAX) {
        why = "need 1 <= m <= 2^31 - 1 and 1 <= n <= 2^31 - 2";
        return false;
    }
    if (A->nnz < A->n || !A->col_ptr || !A->row_idx || !A->values) {
        why = "nnz must be >= n and arrays non-NULL";
        return false;
    }
    if (tau < 1 || tau > A->n) {
        why = "need 1 <= tau <= n";
        return false;
    }
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) {
        why = "lambda must be finite and >= 0";
        return false;
    }
    return true;
}

int batch_create_impl(int count, const pcdm_csc *A, const double *const *b, const double *lambda,
                      const int64_t *tau, uint64_t seed, pcdm_batch **out)
{
    if (!out)
        return fail(PCDM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !A || !b || !lambda || !tau)
        return fail(PCDM_EINVAL, "need count >= 1 and non-NULL arrays");
    const int dtype = A[0].dtype;
    const int on_device = A[0].on_device;
    if (value_bytes(dtype) == 0)
        return fail(PCDM_EINVAL, "unknown dtype");
    for (int j = 0; j < count; ++j) {
        std::string why;
        if (!valid_instance(&A[j], lambda[j], tau[j], why))
            return fail(PCDM_EINVAL, "problem " + std::to_string(j) + ": " + why);
        if (A[j].dtype != dtype || A[j].on_device != on_device || !b[j])
            return fail(PCDM_EINVAL, "problem " + std::to_string(j) + ": every problem needs the same dtype and "
                                     "memory kind, and a b array");
        if ((uint64_t)A[j].m * (dtype == PCDM_F64 ? 8u : 4u) >= (1ull << 32))
            return fail(PCDM_EINVAL, "problem " + std::to_string(j) + ": residual must span < 4 GiB");
    }
    pcdm_batch *B = new (std::nothrow) pcdm_batch();
    if (!B)
        return fail(PCDM_ENOMEM, "host allocation failed");
    struct Guard {
        pcdm_batch *p;
        DevTemps tmp;
        ~Guard() { batch_free(p); }
    } guard{B, {}};
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    B->nblk_max = std::max(64, cus * 8);
    B->count = count;
    B->dtype = dtype;
    B->vb = value_bytes(dtype);
    B->tbytes = dtype == PCDM_F64 ? 8 : 4;
    B->seed = seed;
    B->hdesc.resize(count);
    B->hactive.assign(count, 1);
    B->omega.assign(count, 0);
    B->stored.assign(count, 0);
    B->k_host.assign(count, 0);
    B->beta.assign(count, 1.0);
    B->lambda.assign(lambda, lambda + count);
    B->atb_inf.assign(count, 0.0);
    hipStream_t s = nullptr;
    const int64_t EB = 4 + (int64_t)B->vb;

    Ctrl *ctrl = nullptr;
    PCDM_TRY(guard.tmp.get(&ctrl, sizeof(Ctrl)));
    int64_t sum_n1 = 0, max_n = 0, max_m = 0, max_nnz = 0;
    for (int j = 0; j < count; ++j) {
        sum_n1 += A[j].n + 1;
        max_n = std::max(max_n, A[j].n);
        max_m = std::max(max_m, A[j].m);
        max_nnz = std::max(max_nnz, A[j].nnz);
    }
    HIP_TRY(hipMalloc(&B->pc_all, (size_t)sum_n1 * 8));
    int64_t *dpad = nullptr, *cp_dev = nullptr;
    int32_t *rows_dev = nullptr, *hist = nullptr;
    void *vals_dev = nullptr, *scan_tmp = nullptr;
    PCDM_TRY(guard.tmp.get(&dpad, (size_t)(max_n + 1) * 8));
    PCDM_TRY(guard.tmp.get(&hist, (size_t)max_m * 4));
    if (!on_device) {
        PCDM_TRY(guard.tmp.get(&cp_dev, (size_t)(max_n + 1) * 8));
        PCDM_TRY(guard.tmp.get(&rows_dev, (size_t)max_nnz * 4));
        PCDM_TRY(guard.tmp.get(&vals_dev, (size_t)max_nnz * B->vb));
    }
    size_t scan_bytes = 0;
    HIP_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, dpad, B->pc_all, (int)(max_n + 1), s));
    PCDM_TRY(guard.tmp.get(&scan_tmp, scan_bytes));

    // pass 1: padded pointers, record sizes, bases
    int64_t pc_base = 0, rec_base = 0, row_base = 0, col_base = 0, slot_base = 0;
    int64_t step_t = 0, col_t = 0, row_t = 0;
    for (int j = 0; j < count; ++j) {
        const pcdm_csc &a = A[j];
        const int64_t *cp = a.col_ptr;
        if (!on_device) {
            HIP_TRY(hipMemcpy(cp_dev, a.col_ptr, (size_t)(a.n + 1) * 8, hipMemcpyHostToDevice));
            cp = cp_dev;
        }
        HIP_TRY(hipMemset(ctrl, 0, sizeof(Ctrl)));
        const int g = grid_for(a.n + 1, kBlock, B->nblk_max);
        hipLaunchKernelGGL(k_check_ptr, dim3(g), dim3(kBlock), 0, s, cp, a.n, a.nnz, dpad, ctrl);
        hipLaunchKernelGGL(k_check_uniform, dim3(g), dim3(kBlock), 0, s, (const int64_t *)dpad, a.n, ctrl);
        PCDM_TRY(check_launch("batch k_check_ptr"));
        Ctrl hc;
        HIP_TRY(hipMemcpy(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err)
            return fail(PCDM_EINVAL, "problem " + std::to_string(j) + ": invalid matrix: " + describe_err(hc.err));
        size_t sb = scan_bytes;
        HIP_TRY(hipcub::DeviceScan::ExclusiveSum(scan_tmp, sb, dpad, B->pc_all + pc_base, (int)(a.n + 1), s));
        HIP_TRY(hipMemcpy(&B->stored[j], B->pc_all + pc_base + a.n, 8, hipMemcpyDeviceToHost));
        BatchInst &d = B->hdesc[j];
        d.lay.pc = B->pc_all + pc_base;
        d.lay.fixed_dpad = 0;
        d.lay.stride = 0;
        if (!hc.nonuniform) {
            HIP_TRY(hipMemcpy(&d.lay.fixed_dpad, dpad, 8, hipMemcpyDeviceToHost));
            d.lay.stride = kHeader + d.lay.fixed_dpad * EB;
        }
        d.rec_base = rec_base;
        d.row_base = row_base;
        d.col_base = col_base;
        d.slot_base = slot_base;
        d.step_tile0 = step_t;
        d.m = a.m;
        d.n = a.n;
        d.tau = tau[j];
        d.spe = ceil_div(a.n, tau[j]);
        d.seed = seed + (uint64_t)j;
        d.k = 0;
        d.lam = lambda[j];
        pc_base += a.n + 1;
        rec_base += B->stored[j] * EB + (int64_t)kHeader * a.n;
        rec_base = (rec_base + 15) & ~(int64_t)15;
        row_base += a.m;
        col_base += a.n;
        slot_base += tau[j];
        step_t += ceil_div(tau[j], 64);
        col_t += ceil_div(a.n, 64);
        row_t += ceil_div(a.m, 64);
    }
    B->n_step_tiles = step_t;
    B->n_col_tiles = col_t;
    B->n_row_tiles = row_t;
    HIP_TRY(hipMalloc(&B->seg, (size_t)rec_base));
    HIP_TRY(hipMalloc(&B->x, (size_t)col_base * 8));
    HIP_TRY(hipMemset(B->x, 0, (size_t)col_base * 8));
    HIP_TRY(hipMalloc(&B->r, (size_t)row_base * B->tbytes));
    HIP_TRY(hipMalloc(&B->r64, (size_t)row_base * 8));
    HIP_TRY(hipMalloc(&B->b, (size_t)row_base * 8));
    HIP_TRY(hipMalloc(&B->id_slot, (size_t)slot_base * 4));
    HIP_TRY(hipMalloc(&B->delta_slot, (size_t)slot_base * B->tbytes));
    HIP_TRY(hipMalloc(&B->desc, sizeof(BatchInst) * count));
    HIP_TRY(hipMalloc(&B->active, 4 * (size_t)count));
    HIP_TRY(hipMalloc(&B->acc, 64 * (size_t)count));
    HIP_TRY(hipMalloc(&B->rold, (size_t)row_base * 8));
    HIP_TRY(hipMemset(B->rold, 0, (size_t)row_base * 8));
    HIP_TRY(hipMalloc(&B->ubc, (size_t)col_base * 4));
    HIP_TRY(hipMalloc(&B->nrmc, (size_t)col_base * 4));
    HIP_TRY(hipMalloc(&B->ist, 32 * (size_t)count));
    HIP_TRY(hipMemset(B->ist, 0, 32 * (size_t)count));
    HIP_TRY(hipMalloc(&B->nz_part, 8 * (size_t)B->nblk_max));
    HIP_TRY(hipMemset(B->nz_part, 0, 8 * (size_t)B->nblk_max));
    {
        std::vector<int32_t> st(step_t);
        for (int j = 0; j < count; ++j) {
            const BatchInst &d = B->hdesc[j];
            for (int64_t t = 0; t < ceil_div(d.tau, 64); ++t) st[d.step_tile0 + t] = j;
        }
        HIP_TRY(hipMalloc(&B->list.n, 4));
        HIP_TRY(hipMalloc(&B->list.ids, 4 * (size_t)count));
        HIP_TRY(hipMalloc(&B->list.colp, 8 * ((size_t)count + 1)));
        HIP_TRY(hipMalloc(&B->list.rowp, 8 * ((size_t)count + 1)));
        HIP_TRY(hipMalloc(&B->step_tiles, 4 * (size_t)step_t));
        HIP_TRY(hipMemcpy(B->step_tiles, st.data(), 4 * (size_t)step_t, hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&B->sel, 4 * (size_t)count));
        B->hsel.assign(count, 1);
        HIP_TRY(hipMemcpy(B->sel, B->hsel.data(), 4 * (size_t)count, hipMemcpyHostToDevice));
        B->cF.assign(count, 0.0);
        B->cG.assign(count, 0.0);
        B->ck.assign(count, -1);
        B->cvalid.assign(count, 0);
        B->inc_evals.assign(count, 0);
        B->cands.assign(count, -1);
        B->inc_state.assign(count, 1);  // set by the evaluation at create
    }

    // pass 2: pack every problem, omega_j, b_j
    for (int j = 0; j < count; ++j) {
        const pcdm_csc &a = A[j];
        const int64_t *cp = a.col_ptr;
        const int32_t *rw = a.row_idx;
        const void *vl = a.values;
        if (!on_device) {
            HIP_TRY(hipMemcpy(cp_dev, a.col_ptr, (size_t)(a.n + 1) * 8, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(rows_dev, a.row_idx, (size_t)a.nnz * 4, hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(vals_dev, a.values, (size_t)a.nnz * B->vb, hipMemcpyHostToDevice));
            cp = cp_dev;
            rw = rows_dev;
            vl = vals_dev;
        }
        HIP_TRY(hipMemset(ctrl, 0, sizeof(Ctrl)));
        HIP_TRY(hipMemset(hist, 0, (size_t)a.m * 4));
        const int gm = grid_for(a.m, kBlock, B->nblk_max);
        int64_t *part = nullptr;
        PCDM_TRY(guard.tmp.get(&part, (size_t)std::max(gm, B->nblk_max) * 8));
        batch_dispatch(dtype, [&](auto ops) {
            decltype(ops)::pack(B, cp, rw, vl, j, hist, ctrl, s);
            decltype(ops)::col_norms(B, j, reinterpret_cast<double *>(part), s);
            return PCDM_OK;
        });
        hipLaunchKernelGGL(k_imax_partials, dim3(gm), dim3(kBlock), 0, s, (const int32_t *)hist, a.m, part);
        hipLaunchKernelGGL(k_imax_final, dim3(1), dim3(kBlock), 0, s, (const int64_t *)part, gm, ctrl);
        PCDM_TRY(check_launch("batch k_pack"));
        Ctrl hc;
        HIP_TRY(hipMemcpy(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
        if (hc.err)
            return fail(PCDM_EINVAL, "problem " + std::to_string(j) + ": invalid matrix: " + describe_err(hc.err));
        B->omega[j] = hc.imax;
        const double om = (double)hc.imax, ta = (double)tau[j], nn = (double)a.n;
        B->beta[j] = 1.0 + (om - 1.0) * (ta - 1.0) / std::max(1.0, nn - 1.0);
        B->hdesc[j].inv_beta = 1.0 / B->beta[j];
        HIP_TRY(hipMemcpy(B->b + B->hdesc[j].row_base, b[j], (size_t)a.m * 8,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(B->desc, B->hdesc.data(), sizeof(BatchInst) * count, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(B->active, B->hactive.data(), 4 * (size_t)count, hipMemcpyHostToDevice));
    {
        // schedule from the mean padded column length over all problems
        int64_t st_all = 0, n_all = 0;
        for (int j = 0; j < count; ++j) {
            st_all += B->stored[j];
            n_all += A[j].n;
        }
        const double chunks = (double)st_all / (4.0 * (double)n_all);
        B->lanes = chunks <= 1.0 ? 1 : chunks <= 2.0 ? 2 : chunks <= 4.0 ? 4 : chunks <= 8.0 ? 8 : chunks <= 16.0 ? 16 : 64;
        B->chunks = 1;
    }
    // r = -b and ||A_j^T b_j||_inf (objective pass at x = 0)
    PCDM_TRY(batch_dispatch(dtype, [&](auto ops) {
        decltype(ops)::objective(B, s);
        decltype(ops)::narrow_all(B, s);
        return PCDM_OK;
    }));
    PCDM_TRY(check_launch("batch init"));
    std::vector<double> acc(4 * (size_t)count);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(acc.data(), B->acc, 32 * (size_t)count, hipMemcpyDeviceToHost));
    for (int j = 0; j < count; ++j)
        B->atb_inf[j] = acc[4 * j + 3];
    guard.p = nullptr;
    *out = B;
    return PCDM_OK;
}

}  // namespace

extern "C" {

int pcdm_batch_create(int count, const pcdm_csc *A, const double *const *b, const double *lambda,
                      const int64_t *tau, uint64_t seed, pcdm_batch **out)
{
    t_err.clear();
    try {
        return batch_create_impl(count, A, b, lambda, tau, seed, out);
    } catch (const std::exception &e) {
        return fail(PCDM_EDEVICE, std::string("exception: ") + e.what());
    } catch (...) {
        return fail(PCDM_EDEVICE, "unknown exception");
    }
}

int pcdm_batch_destroy(pcdm_batch *B)
{
    if (!B)
        return PCDM_OK;
    hipError_t e = hipDeviceSynchronize();
    batch_free(B);
    if (e != hipSuccess)
        return hip_fail(e, "pcdm_batch_destroy");
    return PCDM_OK;
}

int pcdm_batch_step(pcdm_batch *B, int64_t nsteps, void *stream)
{
    if (!B)
        return fail(PCDM_EINVAL, "NULL handle");
    if (nsteps < 0)
        return fail(PCDM_EINVAL, "nsteps must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    int64_t left = nsteps;
    if (B->graph_len > 0 && nsteps >= B->graph_len) {
        if (!B->exec || B->graph_captured_len != B->graph_len)
            PCDM_TRY(batch_capture(B));
        for (; left >= B->graph_len; left -= B->graph_len)
            HIP_TRY(hipGraphLaunch(B->exec, s));
    }
    for (; left > 0; --left)
        PCDM_TRY(batch_step_direct(B, s));
    for (int j = 0; j < B->count; ++j)
        if (B->hactive[j])
            B->k_host[j] += nsteps;
    return check_launch("pcdm_batch_step");
}

int pcdm_batch_objective(pcdm_batch *B, double *F, double *gap, void *stream)
{
    if (!B || !F)
        return fail(PCDM_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    // Evaluate the problems that stepped since their last evaluation (or never
    // had one); the others have not changed and keep their values.
    bool any = false;
    for (int j = 0; j < B->count; ++j) {
        B->hsel[j] = (!B->cvalid[j] || B->ck[j] != B->k_host[j]) ? 1 : 0;
        any = any || B->hsel[j];
    }
    std::vector<double> acc(8 * (size_t)B->count, 0.0);
    if (any) {
        HIP_TRY(hipMemcpyAsync(B->sel, B->hsel.data(), 4 * (size_t)B->count, hipMemcpyHostToDevice, s));
        PCDM_TRY(batch_dispatch(B->dtype, [&](auto ops) {
            decltype(ops)::objective(B, s);
            return PCDM_OK;
        }));
        PCDM_TRY(check_launch("pcdm_batch_objective"));
        HIP_TRY(hipMemcpyAsync(acc.data(), B->acc, 64 * (size_t)B->count, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    for (int j = 0; j < B->count; ++j) {
        if (B->hsel[j]) {
            const double rr = acc[4 * j], br = acc[4 * j + 1], l1 = acc[4 * j + 2], gm = acc[4 * j + 3];
            const double lam = B->lambda[j];
            const double Fj = 0.5 * rr + lam * l1;
            const double sc = gm > lam ? lam / gm : 1.0;
            B->cF[j] = Fj;
            B->cG[j] = Fj - (-0.5 * sc * sc * rr - sc * br);
            B->ck[j] = B->k_host[j];
            B->cvalid[j] = 1;
            B->cands[j] = (int64_t)acc[4 * (size_t)B->count + 4 * j + 2];
            if (B->incremental && B->inc_state[j])
                B->inc_evals[j]++;
        }
        F[j] = B->cF[j];
        if (gap)
            gap[j] = B->cG[j];
    }
    return PCDM_OK;
}

int pcdm_batch_set_active(pcdm_batch *B, const int32_t *active)
{
    if (!B || !active)
        return fail(PCDM_EINVAL, "NULL argument");
    for (int j = 0; j < B->count; ++j)
        B->hactive[j] = active[j] ? 1 : 0;
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(B->active, B->hactive.data(), 4 * (size_t)B->count, hipMemcpyHostToDevice));
    return PCDM_OK;
}

int pcdm_batch_get_x(pcdm_batch *B, int index, double *x_out, int32_t on_device, void *stream)
{
    if (!B || !x_out || index < 0 || index >= B->count)
        return fail(PCDM_EINVAL, "bad handle, index or output");
    hipStream_t s = (hipStream_t)stream;
    const BatchInst &d = B->hdesc[index];
    HIP_TRY(hipMemcpyAsync(x_out, B->x + d.col_base, (size_t)d.n * 8,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    if (!on_device)
        HIP_TRY(hipStreamSynchronize(s));
    return PCDM_OK;
}

int pcdm_batch_get_info(pcdm_batch *B, int index, pcdm_info *out)
{
    if (!B || !out || index < 0 || index >= B->count)
        return fail(PCDM_EINVAL, "bad handle, index or output");
    const BatchInst &d = B->hdesc[index];
    std::memset(out, 0, sizeof(*out));
    out->m = d.m;
    out->n = d.n;
    out->tau = d.tau;
    out->k = B->k_host[index];
    out->omega = B->omega[index];
    out->refresh_every = d.spe;
    out->stored_nnz = B->stored[index];
    out->beta = B->beta[index];
    out->lambda = B->lambda[index];
    out->sampling = 0;  // batches use the tau-nice sampler
    out->binomial_p = 1.0;
    out->expected_set_size = (double)d.tau;
    out->atb_inf = B->atb_inf[index];
    out->dtype = B->dtype;
    out->lanes_per_column = B->lanes;
    out->chunks_per_lane = B->chunks;
    out->nonzero_updates = -1;  // not tracked per problem
    out->max_incremental = B->inc_evals[index];
    out->max_candidates = B->cands[index];
    return PCDM_OK;
}

int pcdm_batch_set_option(pcdm_batch *B, const char *key, double value)
{
    if (!B || !key)
        return fail(PCDM_EINVAL, "NULL handle or key");
    const std::string k(key);
    const int v = (int)value;
    if (!std::isfinite(value) || (double)v != value || v < 0)
        return fail(PCDM_EINVAL, "option value must be a non-negative integer");
    if (k == "graph_steps") {
        B->graph_len = v;
        batch_drop_graph(B);
    } else if (k == "max_passes") {
        if (v < 1 || v > 3)
            return fail(PCDM_EINVAL, "max_passes must be 1, 2 or 3");
        B->incremental = v == 3;
    } else if (k == "lanes_per_column" || k == "chunks_per_lane") {
        const int g = k == "lanes_per_column" ? v : B->lanes;
        const int c = k == "chunks_per_lane" ? v : (schedule_supported(v, B->chunks) ? B->chunks : 1);
        if (!schedule_supported(g, c))
            return fail(PCDM_EINVAL, "unsupported (lanes_per_column, chunks_per_lane) pair");
        B->lanes = g;
        B->chunks = c;
        batch_drop_graph(B);
    } else {
        return fail(PCDM_EINVAL, "unknown option '" + k + "'");
    }
    return PCDM_OK;
}

int pcdm_batch_autotune(pcdm_batch *B, int64_t steps_per_candidate, void *stream)
{
    if (!B || steps_per_candidate < 1)
        return fail(PCDM_EINVAL, "NULL handle or steps_per_candidate < 1");
    hipStream_t s = (hipStream_t)stream;
    static const int cand[][2] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {4, 1}, {4, 2}, {8, 1}, {16, 1}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = std::numeric_limits<float>::max();
    int bg = B->lanes, bc = B->chunks;
    int st = PCDM_OK;
    for (const auto &c : cand) {
        B->lanes = c[0];
        B->chunks = c[1];
        (void)hipEventRecord(e0, s);
        for (int64_t q = 0; q < steps_per_candidate && st == PCDM_OK; ++q)
            st = batch_step_direct(B, s);
        (void)hipEventRecord(e1, s);
        if (st != PCDM_OK)
            break;
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            break;
        if (ms < best) {
            best = ms;
            bg = c[0];
            bc = c[1];
        }
        for (int j = 0; j < B->count; ++j)
            if (B->hactive[j])
                B->k_host[j] += steps_per_candidate;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->lanes = bg;
    B->chunks = bc;
    batch_drop_graph(B);
    return st;
}

}  // extern "C"

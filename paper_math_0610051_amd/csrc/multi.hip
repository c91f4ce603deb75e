// Multi-instance apply (instances of uneven N, each its own plan): the three
// stages run as one launch each over the union of every instance's work items
// (box rows, column groups x right-hand sides, output tiles), and that launch
// sequence is captured into a HIP graph.  The graph and the device tables are
// cached in the first plan and replayed while the instance list (plans and
// batch sizes) stays the same; new data pointers only refresh the argument
// table.  Instances of different kernel widths share the launch of the
// widest width, whose interpolation records the windows of every instance
// when the state is built.  Instance lists the fused path cannot take (mixed factor
// modes, a batch larger than a plan's workspace, or one plan listed twice,
// whose single workspace cannot hold two instances at once) run instance
// after instance.
#include <algorithm>
#include <cstring>
#include <vector>

#include "apply.hpp"
#include "errors.hpp"
#include "multi.hpp"

namespace fio {

struct MultiState {
    std::vector<unsigned long long> serials;
    std::vector<int> B;
    std::vector<const void *> f;
    std::vector<void *> u;
    MultiLaunch ml;
    void *d_inst = nullptr;
    MultiRowItem *d_rows = nullptr;
    MultiColItem *d_cols = nullptr;
    MultiTile *d_tiles = nullptr;
    WinRec *d_win = nullptr;           // every instance's window table, recorded by the fused kernel
    std::vector<long long> win_off;    // first record of instance i
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // recorded after each replay, on the caller's stream
    bool launched = false;
    ~MultiState() {
        if (done)
            (void)hipEventDestroy(done);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (cap)
            (void)hipStreamDestroy(cap);
        void *bufs[] = {d_inst, d_rows, d_cols, d_tiles, d_win};
        for (void *b : bufs)
            if (b)
                (void)hipFree(b);
    }
};

void multi_release(fio_plan_s *P) {
    delete static_cast<MultiState *>(P->multi_state);
    P->multi_state = nullptr;
}

static fio_status run_sequential(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u,
                                 const int *B, hipStream_t s) {
    for (int i = 0; i < n; ++i)
        FIO_HIP_TRY(apply_launch(plans[i], B[i], fhat[i], u[i], s, 0, plans[i]->L));
    return FIO_OK;
}

static fio_status build_state(MultiState &st, int n, const fio_plan_t *plans, const int *B) {
    std::vector<MultiRowItem> rows;
    std::vector<MultiColItem> cols;
    std::vector<MultiTile> tiles;
    size_t lds_rows = 0, lds_cols = 0;
    // heaviest instances first (wedge count x grid points x batch), so the
    // launch does not end on a tail of long workgroups
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double wx = (double)plans[x]->L * plans[x]->N * plans[x]->N * B[x];
        const double wy = (double)plans[y]->L * plans[y]->N * plans[y]->N * B[y];
        return wx > wy;
    });
    for (int i : order) {
        const fio_plan_s *P = plans[i];
        for (const RowItem &r : P->rows)
            rows.push_back(MultiRowItem{i, r});
        for (int b = 0; b < B[i]; ++b)
            for (const ColItem &c : P->cols)
                cols.push_back(MultiColItem{i, b, c});
        lds_rows = std::max(lds_rows, P->lds_rows);
        lds_cols = std::max(lds_cols, P->lds_cols);
    }
    // Interpolation tiles, in groups of up to kInterpBatch right-hand sides.
    // Workgroup i of a launch runs on die i % kXcds.  Each instance's tiles are
    // cut into runs of 64 along the chunked walk (8 x 8-tile squares); the runs
    // are dealt, heaviest instance first, to the die stream of least work so
    // far (work ~ wedges x right-hand sides per tile), and the streams are
    // interleaved so that slot i holds die i % kXcds's next tile: each die
    // then walks whole squares (the halos of neighbouring tiles meet in its
    // L2) while the dies get equal work.  Streams that run out are padded
    // with empty entries (nb = 0).
    {
        std::vector<std::vector<MultiTile>> stream(kXcds);
        std::vector<double> work(kXcds, 0.0);
        for (int i : order) {
            const fio_plan_s *P = plans[i];
            const int t = (P->N + kTileX - 1) / kTileX;
            for (int b0 = 0; b0 < B[i]; b0 += kInterpBatch) {
                const int nb = std::min(kInterpBatch, B[i] - b0);
                for (int k0 = 0; k0 < t * t; k0 += 64) {
                    const int k1 = std::min(t * t, k0 + 64);
                    const int x = (int)(std::min_element(work.begin(), work.end()) - work.begin());
                    for (int k = k0; k < k1; ++k)
                        stream[x].push_back(MultiTile{i, chunked_tile(k, t), b0, nb});
                    work[x] += (double)(k1 - k0) * P->L * nb;
                }
            }
        }
        size_t longest = 0;
        for (const auto &v : stream)
            longest = std::max(longest, v.size());
        for (size_t k = 0; k < longest; ++k)
            for (int x = 0; x < kXcds; ++x)
                tiles.push_back(k < stream[x].size() ? stream[x][k] : MultiTile{0, 0, 0, 0});
    }
    const size_t isz = inst_args_size(plans[0]->precision);
    FIO_HIP_TRY(hipMalloc(&st.d_inst, isz * n));
    FIO_HIP_TRY(hipMalloc(&st.d_rows, sizeof(MultiRowItem) * std::max<size_t>(1, rows.size())));
    FIO_HIP_TRY(hipMalloc(&st.d_cols, sizeof(MultiColItem) * std::max<size_t>(1, cols.size())));
    FIO_HIP_TRY(hipMalloc(&st.d_tiles, sizeof(MultiTile) * std::max<size_t>(1, tiles.size())));
    FIO_HIP_TRY(hipMemcpy(st.d_rows, rows.data(), sizeof(MultiRowItem) * rows.size(), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(st.d_cols, cols.data(), sizeof(MultiColItem) * cols.size(), hipMemcpyHostToDevice));
    FIO_HIP_TRY(hipMemcpy(st.d_tiles, tiles.data(), sizeof(MultiTile) * tiles.size(), hipMemcpyHostToDevice));
    st.ml.precision = plans[0]->precision;
    // one interpolation kernel of the widest stencil serves every instance:
    // an instance of width w < W computes its weights with its own w and
    // beta, which vanish beyond w/2, so the extra taps add exact zeros
    st.ml.w = 0;
    for (int i = 0; i < n; ++i)
        st.ml.w = std::max(st.ml.w, plans[i]->w);
    st.ml.inst = st.d_inst;
    st.ml.rows = st.d_rows;
    st.ml.cols = st.d_cols;
    st.ml.tiles = st.d_tiles;
    st.ml.nrows = (unsigned)rows.size();
    st.ml.ncols = (unsigned)cols.size();
    st.ml.ntiles = (unsigned)tiles.size();
    st.ml.lds_rows = lds_rows;
    st.ml.lds_cols = lds_cols;
    st.ml.regen = plans[0]->regen;
    // the largest window + gamma^x an instance uses
    for (int i = 0; i < n; ++i) {
        const int q = plans[i]->qmax;
        const size_t b = plans[i]->precision == FIO_F64
                             ? (size_t)interp_window_bytes<double>(q) + interp_gx_lds_bytes<double>(q)
                             : (size_t)interp_window_bytes<float>(q) + interp_gx_lds_bytes<float>(q);
        st.ml.lds_interp = std::max(st.ml.lds_interp, b);
    }
    // the fused interpolation records every instance's windows once (a
    // launch of it alone, no right-hand sides written); its replays read them
    {
        long long total = 0;
        st.win_off.assign(n, 0);
        for (int i = 0; i < n; ++i) {
            const long long t = (plans[i]->N + kTileX - 1) / kTileX;
            st.win_off[i] = total;
            total += t * t * plans[i]->L;
        }
        FIO_HIP_TRY(hipMalloc(&st.d_win, sizeof(WinRec) * (size_t)std::max<long long>(1, total)));
        const size_t isz = inst_args_size(plans[0]->precision);
        std::vector<unsigned char> host(isz * n);
        for (int i = 0; i < n; ++i)
            fill_inst_args(plans[i], nullptr, nullptr, 0, st.d_win + st.win_off[i], kWinRecord, host.data() + isz * i);
        FIO_HIP_TRY(hipMemcpy(st.d_inst, host.data(), host.size(), hipMemcpyHostToDevice));
        FIO_HIP_TRY(multi_record_windows(st.ml, 0));
        FIO_HIP_TRY(hipStreamSynchronize(0));
    }
    FIO_HIP_TRY(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    // capture the three launches once
    FIO_HIP_TRY(hipStreamCreateWithFlags(&st.cap, hipStreamNonBlocking));
    FIO_HIP_TRY(hipStreamBeginCapture(st.cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = multi_launch(st.ml, st.cap);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(st.cap, &graph);
    if (le != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return hip_fail(le, "multi-instance launch during capture");
    }
    FIO_HIP_TRY(ce);
    hipError_t ie = hipGraphInstantiate(&st.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    FIO_HIP_TRY(ie);
    return FIO_OK;
}

fio_status multi_apply(int n, const fio_plan_t *plans, const void *const *fhat, void *const *u, const int *B,
                       hipStream_t s) {
    bool fused = true;
    for (int i = 0; i < n; ++i)
        if (plans[i]->regen != plans[0]->regen || B[i] > plans[i]->bchunk)
            fused = false;
    // a plan listed twice would have both instances in its one workspace at once
    for (int i = 0; fused && i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                fused = false;
    if (!fused)
        return run_sequential(n, plans, fhat, u, B, s);
    fio_plan_s *owner = plans[0];
    MultiState *st = static_cast<MultiState *>(owner->multi_state);
    bool same = st && (int)st->serials.size() == n;
    for (int i = 0; same && i < n; ++i)
        same = st->serials[i] == plans[i]->serial && st->B[i] == B[i];
    if (!same) {
        multi_release(owner);
        st = new MultiState();
        owner->multi_state = st;
        for (int i = 0; i < n; ++i) {
            st->serials.push_back(plans[i]->serial);
            st->B.push_back(B[i]);
        }
        fio_status bs = build_state(*st, n, plans, B);
        if (bs != FIO_OK) {
            multi_release(owner);
            return bs;
        }
        st->f.assign(n, nullptr);
        st->u.assign(n, nullptr);
    }
    bool ptrs = true;
    for (int i = 0; i < n; ++i)
        ptrs = ptrs && st->f[i] == fhat[i] && st->u[i] == u[i];
    if (!ptrs) {
        // the previous replay, on whichever stream it ran, may still read the
        // argument table: wait for it before the table is overwritten
        if (st->launched)
            FIO_HIP_TRY(hipEventSynchronize(st->done));
        const size_t isz = inst_args_size(owner->precision);
        std::vector<unsigned char> host(isz * n);
        for (int i = 0; i < n; ++i) {
            fill_inst_args(plans[i], fhat[i], u[i], B[i], st->d_win + st->win_off[i], kWinUse, host.data() + isz * i);
            st->f[i] = fhat[i];
            st->u[i] = u[i];
        }
        FIO_HIP_TRY(hipMemcpy(st->d_inst, host.data(), host.size(), hipMemcpyHostToDevice));
    }
    FIO_HIP_TRY(hipGraphLaunch(st->exec, s));
    FIO_HIP_TRY(hipEventRecord(st->done, s));
    st->launched = true;
    return FIO_OK;
}

}  // namespace fio

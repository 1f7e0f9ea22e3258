/*
 * A plain C caller of the library's C ABI (include/lc.h), with no Python in
 * the process: the sequence of Sec. 2.2's algorithm as the boundary exposes
 * it. Step 1 is lc_plan (the box, the grid and the lookback shells), steps
 * 2-3 are lc_build_greens, step 4 is lc_push_sources per slice and steps
 * 5-6 are lc_field.
 *
 * Usage: c_abi_example <input> <output> <precision>
 *   input:  int32 n, int32 K, int32 m, double L, double radii[K+1], then per
 *           slice int64 count, int64 cells[count], double lum[count]
 *   output: two fields, N^3 doubles each in the grid layout of lc.h: first
 *           from host point lists pushed slice by slice and lc_field into
 *           host memory; then from one whole step (lc_step) over dense
 *           device grids into device memory, replayed from its captured
 *           HIP graph (the second of two steps)
 *   precision: an lc_precision value
 * Device memory (the workspace, the dense grids, the step's output) comes
 * from the HIP runtime. Exit status 0 on success; on failure the library's
 * message is printed.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "lc.h"

static int fail(const char *what, int rc) {
    fprintf(stderr, "%s failed (%d): %s\n", what, rc, lc_last_error());
    return 1;
}

static int read_all(FILE *f, void *p, size_t size, size_t count) {
    return fread(p, size, count, f) == count;
}

int main(int argc, char **argv) {
    if (argc != 4) {
        fprintf(stderr, "usage: %s <input> <output> <precision>\n", argv[0]);
        return 2;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) {
        perror(argv[1]);
        return 2;
    }
    int32_t n = 0, K = 0, m = 0;
    double L = 0.0;
    if (!read_all(in, &n, 4, 1) || !read_all(in, &K, 4, 1) || !read_all(in, &m, 4, 1) ||
        !read_all(in, &L, 8, 1) || n < 1 || K < 1) {
        fprintf(stderr, "bad input header\n");
        return 2;
    }
    double *radii = malloc(sizeof(double) * (size_t)(K + 1));
    int64_t *counts = calloc((size_t)K, sizeof(int64_t));
    int64_t **cells = calloc((size_t)K, sizeof(int64_t *));
    double **lums = calloc((size_t)K, sizeof(double *));
    if (!radii || !counts || !cells || !lums || !read_all(in, radii, 8, (size_t)(K + 1))) {
        fprintf(stderr, "bad input radii\n");
        return 2;
    }
    for (int k = 0; k < K; ++k) {
        if (!read_all(in, &counts[k], 8, 1) || counts[k] < 0) {
            fprintf(stderr, "bad count of slice %d\n", k);
            return 2;
        }
        cells[k] = malloc(sizeof(int64_t) * (size_t)(counts[k] + 1));
        lums[k] = malloc(sizeof(double) * (size_t)(counts[k] + 1));
        if (!cells[k] || !lums[k] || !read_all(in, cells[k], 8, (size_t)counts[k]) ||
            !read_all(in, lums[k], 8, (size_t)counts[k])) {
            fprintf(stderr, "bad sources of slice %d\n", k);
            return 2;
        }
        for (int64_t i = 0; i < counts[k]; ++i)
            if (cells[k][i] < 0 || cells[k][i] >= (int64_t)n * n * n) {
                fprintf(stderr, "cell out of range in slice %d\n", k);
                return 2;
            }
    }
    fclose(in);

    const size_t n3 = (size_t)n * n * n;
    lc_box_desc box = {0};
    box.n = n;
    box.n_slices = K;
    box.n_bands = 1;
    box.supersample = m;
    box.box = L;
    box.radii = radii;
    lc_plan_desc desc = {0};
    desc.n_boxes = 1;
    desc.precision = atoi(argv[3]);
    desc.boxes = &box;
    desc.use_graph = 1;
    /* a stream of its own (default priority): a graph cannot be captured on
     * the legacy default stream */
    hipStream_t stream = NULL;
    if (hipStreamCreate(&stream) != hipSuccess) {
        fprintf(stderr, "hipStreamCreate failed\n");
        return 1;
    }
    desc.hip_stream = stream;

    const size_t bytes = lc_workspace_bytes(&desc);
    if (bytes == 0) return fail("lc_workspace_bytes", LC_EINVAL);
    void *ws = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    desc.workspace = ws;
    desc.workspace_bytes = bytes;
    lc_plan_t *plan = NULL;
    int rc = lc_plan(&desc, &plan);
    if (rc) return fail("lc_plan", rc);

    lc_atten flat = {0};      /* phi = 1, bare 1/(4 pi r^2) dilution */
    flat.prefactor = 1.0;
    if ((rc = lc_build_greens(plan, 0, 0, &flat))) return fail("lc_build_greens", rc);

    for (int k = 0; k < K; ++k) {
        lc_sources s = {0};
        s.kind = 1;
        s.dtype = LC_F64;
        s.mem = LC_MEM_HOST;
        s.n = counts[k];
        s.cell = cells[k];
        s.lum = lums[k];
        if ((rc = lc_push_sources(plan, 0, k, &s))) return fail("lc_push_sources", rc);
    }

    double *J = malloc(sizeof(double) * 2 * n3);
    if (!J) return 2;
    void *outs[1] = {J};
    if ((rc = lc_field(plan, 0, 0, outs, LC_F64, LC_MEM_HOST))) return fail("lc_field", rc);

    /* the same sources as dense device grids (nearest-grid-point deposit on
     * the host), then two whole steps: the first captures the graph, the
     * second replays it */
    const int grid_f64 = desc.precision == LC_PREC_FP64;
    const size_t vsz = grid_f64 ? sizeof(double) : sizeof(float);
    void *host_grid = calloc(n3, vsz), *dgrids = NULL, *dout = NULL;
    lc_sources *srcs = calloc((size_t)K, sizeof(lc_sources));
    if (!host_grid || !srcs) return 2;
    if (hipMalloc(&dgrids, vsz * n3 * (size_t)K) != hipSuccess || hipMalloc(&dout, sizeof(double) * n3) != hipSuccess) {
        fprintf(stderr, "hipMalloc of the step buffers failed\n");
        return 1;
    }
    for (int k = 0; k < K; ++k) {
        double *g64 = host_grid;
        float *g32 = host_grid;
        for (size_t c = 0; c < n3; ++c) {
            if (grid_f64) g64[c] = 0.0;
            else g32[c] = 0.0f;
        }
        for (int64_t i = 0; i < counts[k]; ++i) {
            if (grid_f64) g64[cells[k][i]] += lums[k][i];
            else g32[cells[k][i]] += (float)lums[k][i];
        }
        char *dst = (char *)dgrids + vsz * n3 * (size_t)k;
        if (hipMemcpy(dst, host_grid, vsz * n3, hipMemcpyHostToDevice) != hipSuccess) return 1;
        srcs[k].kind = 0;
        srcs[k].dtype = grid_f64 ? LC_F64 : LC_F32;
        srcs[k].mem = LC_MEM_DEVICE;
        srcs[k].grid = dst;
    }
    void *douts[1] = {dout};
    for (int rep = 0; rep < 2; ++rep)
        if ((rc = lc_step(plan, srcs, douts, LC_F64))) return fail("lc_step", rc);
    if (hipStreamSynchronize(stream) != hipSuccess ||
        hipMemcpy(J + n3, dout, sizeof(double) * n3, hipMemcpyDeviceToHost) != hipSuccess) {
        fprintf(stderr, "copying the step's field back failed\n");
        return 1;
    }
    lc_destroy(plan);
    hipFree(dgrids);
    hipFree(dout);
    hipFree(ws);
    hipStreamDestroy(stream);
    free(host_grid);
    free(srcs);

    FILE *out = fopen(argv[2], "wb");
    if (!out || fwrite(J, sizeof(double), 2 * n3, out) != 2 * n3) {
        perror(argv[2]);
        return 2;
    }
    fclose(out);
    for (int k = 0; k < K; ++k) {
        free(cells[k]);
        free(lums[k]);
    }
    free(cells);
    free(lums);
    free(counts);
    free(radii);
    free(J);
    return 0;
}

// Runs the emulated library on one input file and writes what it returns.
//
//   driver kmeans in.bin out.bin
//     in:  int64 n, d, k, iters, algo, leaf_size, flags | cand_tile << 20, point_dtype;
//          points (n x d, FP32 or FP64 per point_dtype); c0 (k x d FP64)
//     out: per step: assignment (n int32), centroids (k x d FP64),
//          statistics (7 int64 + 1 double, the km_iter_stats layout)
//   driver run in.bin out.bin            (same input; one kmeans_run call
//          with stop_when_stable = flags >> 16 & 1, max_iter = iters)
//     out: int32 iterations, assignment (n int32), centroids (k x d FP64)
//   driver batched in.bin out.bin        (B clouds in one context: after the
//          header, int64 B, pt_offs (B + 1), c_offs (B + 1); k is c_offs[B])
//     out: as kmeans, with cloud-local assignments
//   driver runb in.bin out.bin           (same input; one kmeans_run_batched
//          call with the header's leaf_size and cand_tile = flags >> 20)
//     out: int32 f, int32 G, assignment (n int32), centroids (k x d FP64)
//   driver info in.bin out.bin / infob   (the input of kmeans / batched; the
//          context is created and released)
//     out: km_ctx_info
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "ekm.h"

static void die(const char *what)
{
    fprintf(stderr, "driver: %s: %s\n", what, kmeans_last_error());
    exit(2);
}

int main(int argc, char **argv)
{
    if (argc != 4) {
        fprintf(stderr, "usage: driver kmeans|run|batched|runb|info|infob in.bin out.bin\n");
        return 2;
    }
    FILE *f = fopen(argv[2], "rb");
    if (!f)
        return 2;
    int64_t h[8];
    if (fread(h, 8, 8, f) != 8)
        return 2;
    const int64_t n = h[0], d = h[1], k = h[2], iters = h[3];
    const bool batched = !strcmp(argv[1], "batched") || !strcmp(argv[1], "runb") || !strcmp(argv[1], "infob");
    const bool info = !strcmp(argv[1], "info") || !strcmp(argv[1], "infob");
    int64_t B = 1;
    std::vector<int64_t> pt_offs, c_offs;
    if (batched) {
        if (fread(&B, 8, 1, f) != 1)
            return 2;
        pt_offs.resize(B + 1);
        c_offs.resize(B + 1);
        if (fread(pt_offs.data(), 8, B + 1, f) != (size_t)(B + 1) ||
            fread(c_offs.data(), 8, B + 1, f) != (size_t)(B + 1))
            return 2;
    }
    const size_t es = h[7] == KM_F32 ? 4 : 8;
    std::vector<unsigned char> pts(n * d * es);
    std::vector<double> c(k * d);
    if (fread(pts.data(), 1, pts.size(), f) != pts.size() || fread(c.data(), 8, c.size(), f) != c.size())
        return 2;
    fclose(f);
    km_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.d = (int32_t)d;
    cfg.point_dtype = (int32_t)h[7];
    cfg.algo = (int32_t)h[4];
    cfg.leaf_size = (int32_t)h[5];
    cfg.flags = (uint32_t)(h[6] & 0xffff);
    cfg.cand_tile = (int32_t)((h[6] >> 20) & 0xfff); // (leaves per list; 0 = default)
    std::vector<int32_t> a(n);
    if (!strcmp(argv[1], "runb")) {
        cfg.flags = 0;
        int32_t tuned[2] = {0, 0};
        if (kmeans_run_batched(pts.data(), pt_offs.data(), c.data(), c_offs.data(), a.data(), (int32_t)B, &cfg,
                               (int32_t)iters, nullptr, tuned) != KM_OK)
            die("kmeans_run_batched");
        FILE *o = fopen(argv[3], "wb");
        fwrite(tuned, 4, 2, o);
        fwrite(a.data(), 4, n, o);
        fwrite(c.data(), 8, c.size(), o);
        fclose(o);
        return 0;
    }
    km_ctx *ctx = nullptr;
    if (batched) {
        if (kmeans_init_batched(&ctx, &cfg, pts.data(), pt_offs.data(), c_offs.data(), (int32_t)B, nullptr) != KM_OK)
            die("kmeans_init_batched");
    } else if (kmeans_init(&ctx, &cfg, pts.data(), n, k, nullptr) != KM_OK)
        die("kmeans_init");
    FILE *o = fopen(argv[3], "wb");
    if (info) {
        km_ctx_info ci;
        if (kmeans_context_info(ctx, &ci) != KM_OK)
            die("kmeans_context_info");
        fwrite(&ci, sizeof(ci), 1, o);
    } else if (!strcmp(argv[1], "kmeans") || batched) {
        std::vector<double> cn(k * d);
        for (int64_t t = 0; t < iters; ++t) {
            km_iter_stats st;
            if (kmeans_step(ctx, c.data(), cn.data(), a.data(), &st) != KM_OK)
                die("kmeans_step");
            fwrite(a.data(), 4, n, o);
            fwrite(cn.data(), 8, cn.size(), o);
            fwrite(&st, sizeof(st), 1, o);
            c.swap(cn);
        }
    } else {
        int32_t it = 0;
        if (kmeans_run(ctx, c.data(), a.data(), (int32_t)iters, (int32_t)((h[6] >> 16) & 1), &it, nullptr) != KM_OK)
            die("kmeans_run");
        fwrite(&it, 4, 1, o);
        fwrite(a.data(), 4, n, o);
        fwrite(c.data(), 8, c.size(), o);
    }
    fclose(o);
    if (kmeans_destroy(ctx) != KM_OK)
        die("kmeans_destroy");
    return 0;
}

// Test driver for the C-ABI without Python or torch: reads a block system
// written by the tests, builds the hierarchy from host-resident blocks, runs a
// V-cycle and a GMRES solve on device vectors it allocates itself, checks
// that aliased V-cycle arguments are rejected, and writes z and x back.
//
//   abi_driver <system.bin> <out.bin> <precision 0|1>
//
// system.bin (little endian): int32 magic 0x4d42414d, n_blocks (2), dofs[0],
// dofs[1], n_vec[0], n_vec[1], then the four blocks A_00, A_01, A_10, A_11,
// each int32 n_brows, n_bcols, br, bc, int64 nnzb, int32 row_ptr[n_brows + 1],
// int32 col_idx[nnzb], float64 vals[nnzb * br * bc]; then int64 n and float64
// b[n].  out.bin: float64 z[n] (V-cycle of b), float64 x[n] (solve of b).
// Prints one line: status, iterations, relative residual, levels.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../include/mbamg.h"

#define HIP_OK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 3;                                                                 \
        }                                                                             \
    } while (0)

template <class T>
static bool read_vec(FILE* f, std::vector<T>& v, size_t n) {
    v.resize(n);
    return n == 0 || std::fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: %s system.bin out.bin precision\n", argv[0]);
        return 2;
    }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t head[6];
    if (std::fread(head, sizeof(int32_t), 6, f) != 6 || head[0] != 0x4d42414d || head[1] != 2) return 2;
    mbamg_field_map fm{};
    fm.n_blocks = 2;
    for (int b = 0; b < 2; ++b) {
        fm.dofs[b] = head[2 + b];
        fm.n_vec[b] = head[4 + b];
    }
    std::vector<int32_t> rp[4], ci[4];
    std::vector<double> val[4];
    mbamg_bsr blocks[4];
    for (int k = 0; k < 4; ++k) {
        int32_t dims[4];
        int64_t nnzb = 0;
        if (std::fread(dims, sizeof(int32_t), 4, f) != 4 || std::fread(&nnzb, sizeof(int64_t), 1, f) != 1) return 2;
        if (!read_vec(f, rp[k], (size_t)dims[0] + 1) || !read_vec(f, ci[k], (size_t)nnzb) ||
            !read_vec(f, val[k], (size_t)nnzb * dims[2] * dims[3]))
            return 2;
        mbamg_bsr& B = blocks[k];
        B.n_brows = dims[0];
        B.n_bcols = dims[1];
        B.br = dims[2];
        B.bc = dims[3];
        B.nnzb = nnzb;
        B.row_ptr = rp[k].data();
        B.col_idx = nnzb ? ci[k].data() : nullptr;
        B.vals = nnzb ? val[k].data() : nullptr;
        B.on_device = 0;
    }
    int64_t n = 0;
    std::vector<double> b;
    if (std::fread(&n, sizeof(int64_t), 1, f) != 1 || !read_vec(f, b, (size_t)n)) return 2;
    std::fclose(f);

    mbamg_params p;
    mbamg_default_params(&p);
    p.precision = std::atoi(argv[3]);
    mbamg_hierarchy* h = nullptr;
    mbamg_status st = mbamg_setup(blocks, &fm, &p, nullptr, &h);
    if (st != MBAMG_OK) {
        std::fprintf(stderr, "setup failed (%d): %s\n", (int)st, mbamg_last_error());
        return 1;
    }
    double *db = nullptr, *dz = nullptr, *dx = nullptr;
    HIP_OK(hipMalloc((void**)&db, sizeof(double) * n));
    HIP_OK(hipMalloc((void**)&dz, sizeof(double) * n));
    HIP_OK(hipMalloc((void**)&dx, sizeof(double) * n));
    HIP_OK(hipMemcpy(db, b.data(), sizeof(double) * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(dx, 0, sizeof(double) * n));
    // aliased arguments are rejected before any kernel runs
    if (mbamg_vcycle(h, db, db, nullptr) != MBAMG_E_INVALID) {
        std::fprintf(stderr, "aliased V-cycle arguments were accepted\n");
        return 1;
    }
    if (mbamg_vcycle(h, db, dz, nullptr) != MBAMG_OK) {
        std::fprintf(stderr, "vcycle failed: %s\n", mbamg_last_error());
        return 1;
    }
    mbamg_info info{};
    st = mbamg_solve(h, db, dx, 1e-8, &info, nullptr);
    std::vector<double> z((size_t)n), x((size_t)n);
    HIP_OK(hipMemcpy(z.data(), dz, sizeof(double) * n, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(x.data(), dx, sizeof(double) * n, hipMemcpyDeviceToHost));
    FILE* o = std::fopen(argv[2], "wb");
    if (!o) return 2;
    std::fwrite(z.data(), sizeof(double), (size_t)n, o);
    std::fwrite(x.data(), sizeof(double), (size_t)n, o);
    std::fclose(o);
    std::printf("status %d iterations %d rel_residual %.6e levels %d\n", (int)st, info.iterations, info.rel_residual,
                info.levels);
    mbamg_destroy(h);
    HIP_OK(hipFree(db));
    HIP_OK(hipFree(dz));
    HIP_OK(hipFree(dx));
    return st == MBAMG_OK ? 0 : 1;
}

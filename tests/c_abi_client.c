/*
 * A C99 program that uses libplanb through include/planb.h alone (no Python,
 * no torch): it reads a rule set and addresses from raw files, resolves every
 * address, and writes the next hops.  The tests compare its output with the
 * oracle's.
 *
 *   c_abi_client MODE PREFIXES LENGTHS HOPS ADDRS OUT
 *     MODE      "host": the host-only halves of the build and the host-core
 *               lookup (planb_build_intervals, planb_build_image,
 *               planb_cpu_lookup); no GPU is touched.
 *               "gpu": planb_build, device buffers from hipMalloc, and
 *               planb_lookup on a HIP stream created here.
 *     PREFIXES  n records of 16 bytes: {uint64 hi, uint64 lo}, native order
 *     LENGTHS   n bytes, 0..128
 *     HOPS      n uint16
 *     ADDRS     k records of 16 bytes, like PREFIXES
 *     OUT       written: k uint16 next hops
 * Exit status 0 on success; otherwise a message on stderr (with
 * planb_last_error() when the library refused a call).
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "planb.h"

static void* slurp(const char* path, size_t* bytes)
{
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* p = malloc(len > 0 ? (size_t)len : 1);
    if (p && len > 0 && fread(p, 1, (size_t)len, f) != (size_t)len) {
        free(p);
        p = NULL;
    }
    fclose(f);
    *bytes = len > 0 ? (size_t)len : 0;
    return p;
}

static int fail(const char* what)
{
    fprintf(stderr, "c_abi_client: %s: %s\n", what, planb_last_error());
    return 1;
}

static int hip_fail(const char* what, hipError_t e)
{
    fprintf(stderr, "c_abi_client: %s: %s\n", what, hipGetErrorString(e));
    return 1;
}

/* Host-only: intervals, the device image, and the host-core descent over it. */
static int run_host(const planb_addr_t* pre, const uint8_t* len, const uint16_t* hop, size_t n,
                    const planb_addr_t* addrs, size_t k, uint16_t* out)
{
    long long m = planb_build_intervals(pre, len, hop, n, 0, NULL, NULL, 0);
    if (m <= 0) return fail("planb_build_intervals");
    planb_addr_t* starts = malloc((size_t)m * sizeof(*starts));
    uint16_t* nh = malloc((size_t)m * sizeof(*nh));
    if (!starts || !nh) return fail("out of host memory");
    if (planb_build_intervals(pre, len, hop, n, 0, starts, nh, (size_t)m) != m) return fail("planb_build_intervals");
    planb_info_t info;
    long long bytes = planb_build_image(starts, nh, (size_t)m, 16, 0, NULL, 0, &info);
    if (bytes <= 0) return fail("planb_build_image");
    void* image = malloc((size_t)bytes);
    if (!image) return fail("out of host memory");
    if (planb_build_image(starts, nh, (size_t)m, 16, 0, image, (size_t)bytes, NULL) != bytes)
        return fail("planb_build_image");
    if (planb_cpu_lookup(image, &info, addrs, k, out, 0) != PLANB_OK) return fail("planb_cpu_lookup");
    free(image);
    free(nh);
    free(starts);
    return 0;
}

/* The GPU path: build, upload, one lookup on a stream of our own, download. */
static int run_gpu(const planb_addr_t* pre, const uint8_t* len, const uint16_t* hop, size_t n,
                   const planb_addr_t* addrs, size_t k, uint16_t* out)
{
    planb_fib_t* fib = planb_build(pre, len, hop, n);
    if (!fib) return fail("planb_build");
    hipStream_t st;
    hipError_t e = hipStreamCreate(&st);
    if (e != hipSuccess) return hip_fail("hipStreamCreate", e);
    planb_addr_t* d_addrs = NULL;
    uint16_t* d_out = NULL;
    if ((e = hipMalloc((void**)&d_addrs, (k ? k : 1) * sizeof(planb_addr_t))) != hipSuccess ||
        (e = hipMalloc((void**)&d_out, (k ? k : 1) * sizeof(uint16_t))) != hipSuccess)
        return hip_fail("hipMalloc", e);
    if ((e = hipMemcpy(d_addrs, addrs, k * sizeof(planb_addr_t), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail("hipMemcpy to the device", e);
    if (planb_lookup(fib, d_addrs, k, d_out, (void*)st) != PLANB_OK) return fail("planb_lookup");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("hipStreamSynchronize", e);
    if ((e = hipMemcpy(out, d_out, k * sizeof(uint16_t), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail("hipMemcpy to the host", e);
    planb_free(fib);
    (void)hipFree(d_out);
    (void)hipFree(d_addrs);
    (void)hipStreamDestroy(st);
    return 0;
}

int main(int argc, char** argv)
{
    if (argc != 7 || (strcmp(argv[1], "host") != 0 && strcmp(argv[1], "gpu") != 0)) {
        fprintf(stderr, "usage: %s host|gpu PREFIXES LENGTHS HOPS ADDRS OUT\n", argv[0]);
        return 2;
    }
    size_t bp, bl, bh, ba;
    planb_addr_t* pre = slurp(argv[2], &bp);
    uint8_t* len = slurp(argv[3], &bl);
    uint16_t* hop = slurp(argv[4], &bh);
    planb_addr_t* addrs = slurp(argv[5], &ba);
    if (!pre || !len || !hop || !addrs) {
        fprintf(stderr, "c_abi_client: cannot read the input files\n");
        return 1;
    }
    const size_t n = bl, k = ba / sizeof(planb_addr_t);
    if (bp != n * sizeof(planb_addr_t) || bh != n * sizeof(uint16_t) || ba % sizeof(planb_addr_t)) {
        fprintf(stderr, "c_abi_client: the input files disagree on the number of rules or records\n");
        return 1;
    }
    uint16_t* out = malloc((k ? k : 1) * sizeof(uint16_t));
    if (!out) return 1;
    int rc = strcmp(argv[1], "host") == 0 ? run_host(pre, len, hop, n, addrs, k, out)
                                          : run_gpu(pre, len, hop, n, addrs, k, out);
    if (rc) return rc;
    FILE* f = fopen(argv[6], "wb");
    if (!f || fwrite(out, sizeof(uint16_t), k, f) != k) {
        fprintf(stderr, "c_abi_client: cannot write %s\n", argv[6]);
        return 1;
    }
    fclose(f);
    printf("c_abi_client %s: %zu rules, %zu addresses resolved\n", argv[1], n, k);
    return 0;
}

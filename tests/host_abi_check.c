/*
 * Host-side check of libzm's C ABI without a GPU, built with the compiler's
 * address / undefined-behaviour sanitizers or its thread sanitizer (see
 * tests/test_sanitize_cpu.py): the pure host functions, the argument checks
 * of every entry point (which must reject null pointers and bad sizes
 * before any device call), and the thread-local error text under several
 * threads calling at once.
 */
#include <pthread.h>
#include <stdio.h>
#include <string.h>

#include "zm.h"

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            __atomic_add_fetch(&fails, 1, __ATOMIC_RELAXED);               \
        }                                                                  \
    } while (0)

static void check_enumeration(int nmax) {
    int idx = 0;
    for (int n = 0; n <= nmax; ++n)
        for (int m = n % 2; m <= n; m += 2) CHECK(zm_index(n, m) == idx++);
    CHECK(zm_num_moments(nmax) == idx);
}

static void check_null_arguments(void) {
    size_t bytes = 0;
    int a = 0, b = 0;
    CHECK(zm_plan_ex(NULL, NULL) == ZM_EINVAL);
    CHECK(zm_plan_info(NULL, NULL) == ZM_EINVAL);
    CHECK(zm_radial_table(NULL, NULL, 0) == ZM_EINVAL);
    CHECK(zm_ring_nodes(NULL, NULL, NULL, 0) == ZM_EINVAL);
    CHECK(zm_operand_table(NULL, NULL, 0) == ZM_EINVAL);
    CHECK(zm_workspace_size(NULL, 1, &bytes) == ZM_EINVAL);
    CHECK(zm_moments(NULL, NULL, 1, 0, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_moments_static(NULL, NULL, 1, 0, NULL, NULL) == ZM_EINVAL);
    CHECK(zm_count_nonfinite(NULL, NULL, 1, NULL, NULL) == ZM_EINVAL);
    CHECK(zm_spectra(NULL, NULL, 1, 0, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_project(NULL, 1, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_moments_polar(NULL, NULL, 1, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_resample_polar(NULL, NULL, 1, 0, NULL, NULL) == ZM_EINVAL);
    CHECK(zm_batch_create(NULL, 0, 0, NULL) == ZM_EINVAL);
    CHECK(zm_batch_run(NULL, NULL) == ZM_EINVAL);
    CHECK(zm_batch_update(NULL, NULL, 0) == ZM_EINVAL);
    CHECK(zm_batch_check(NULL) == ZM_EINVAL);
    CHECK(zm_batch_config(NULL, NULL, NULL, NULL, NULL) == ZM_EINVAL);
    CHECK(zm_batch_destroy(NULL) == ZM_EINVAL);
    CHECK(zm_moments_batch(NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_batch_workspace_size(NULL, 0, &bytes) == ZM_EINVAL);
    CHECK(zm_moments_batch_ws(NULL, 0, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_batch_stage_size(NULL, 0, &bytes) == ZM_EINVAL);
    CHECK(zm_moments_batch_async(NULL, 0, NULL, 0, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_batch_stage_status(NULL) == ZM_EINVAL);
    CHECK(zm_reconstruct(NULL, NULL, 1, NULL, 0, 0, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_recon_workspace_size(NULL, 1, &bytes) == ZM_EINVAL);
    CHECK(zm_recon_error(NULL, NULL, NULL, 1, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_pad_size(0, &a, &b) == ZM_EINVAL);
    CHECK(zm_pad_size(5, NULL, &b) == ZM_EINVAL);
    CHECK(zm_embed(NULL, 4, 1, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_cartesian_workspace_size(0, 1, &bytes) == ZM_EINVAL);
    CHECK(zm_moment_cartesian(NULL, 4, 1, 16, 0, 0, 0, NULL, NULL, 0, NULL) == ZM_EINVAL);
    CHECK(zm_destroy(NULL) == ZM_EINVAL);
    /* a descriptor that fails its checks before any device call */
    zm_plan_desc d;
    memset(&d, 0, sizeof d);
    d.n_max = 20;
    d.H = 64;
    d.W = 64;
    d.dtype = ZM_F32;
    d.angles = 40; /* not a power of two */
    d.device = -1;
    zm_plan_t p = NULL;
    CHECK(zm_plan_ex(&d, &p) == ZM_EINVAL && p == NULL);
    d.angles = 0;
    d.n_max = 501;
    CHECK(zm_plan_ex(&d, &p) == ZM_EINVAL && p == NULL);
    /* frames of 2^31 bytes or more are rejected (32-bit pixel offsets) */
    d.n_max = 20;
    d.H = 16384;
    d.W = 32768;
    CHECK(zm_plan_ex(&d, &p) == ZM_EINVAL && p == NULL);
    d.W = 16384;
    d.dtype = ZM_F64;
    CHECK(zm_plan_ex(&d, &p) == ZM_EINVAL && p == NULL);
}

static void* worker(void* arg) {
    const long id = (long)arg;
    for (int it = 0; it < 300; ++it) {
        const int nmax = (int)((id * 37 + it) % 120);
        CHECK(zm_num_moments(nmax) == (nmax % 2 == 0 ? (nmax / 2 + 1) * (nmax / 2 + 1)
                                                     : (nmax / 2 + 1) * (nmax / 2 + 2)));
        CHECK(zm_index(nmax, nmax) == zm_num_moments(nmax) - 1);
        int size = 0, off = 0;
        CHECK(zm_pad_size(256, &size, &off) == ZM_OK && size == 382 && off == 63);
        /* each thread leaves its own error text and must read back its own */
        if (id % 2 == 0) {
            CHECK(zm_destroy(NULL) == ZM_EINVAL);
            CHECK(strstr(zm_last_error(), "null plan") != NULL);
        } else {
            CHECK(zm_pad_size(-1, &size, &off) == ZM_EINVAL);
            CHECK(strstr(zm_last_error(), "n must be") != NULL);
        }
    }
    return NULL;
}

int main(void) {
    for (int nmax = 0; nmax <= 260; nmax += 13) check_enumeration(nmax);
    check_enumeration(500);
    CHECK(zm_num_moments(-1) == -1);
    CHECK(zm_index(3, 2) == -1 && zm_index(2, 3) == -1 && zm_index(-1, 0) == -1 && zm_index(4, -2) == -1);
    for (int s = 0; s >= -5; --s) CHECK(strncmp(zm_status_str((zm_status)s), "ZM_", 3) == 0);
    CHECK(zm_static_scratch_bytes() == ((size_t)32 << 20));
    check_null_arguments();
    pthread_t th[8];
    for (long i = 0; i < 8; ++i) pthread_create(&th[i], NULL, worker, (void*)i);
    for (int i = 0; i < 8; ++i) pthread_join(th[i], NULL);
    printf("host_abi_check: %d failure(s)\n", fails);
    return fails != 0;
}

/*
 * Runs the threaded PARemSP of the oracle (one POSIX thread per row chunk,
 * boundary unions concurrent under Algorithm 8's locks) under
 * ThreadSanitizer (built by tests/test_oracle_tsan.py with gcc; host code
 * only) and compares every result with the single-threaded CCLRemSP.
 *
 * Images: random binary images of several shapes and densities (dense noise
 * makes many boundary unions land on the same large sets, so threads race
 * for the same roots), horizontal bars crossing every chunk boundary, and a
 * comb whose teeth end at the boundaries; 4- and 8-connectivity; 2 to 16
 * threads.  A data race makes ThreadSanitizer report and exit non-zero; a
 * wrong labeling prints the case and counts as a failure.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_cclremsp(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn, int32_t *labels);
int64_t oracle_paremsp_threads(const uint8_t *img, int64_t H, int64_t W, int64_t stride, int conn,
                               int32_t *labels, int nthreads);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (uint32_t)(rng_state >> 16);
}

static int check(const uint8_t *img, int H, int W, int conn, int threads, const char *what)
{
    int32_t *a = malloc(sizeof(int32_t) * (size_t)H * W), *b = malloc(sizeof(int32_t) * (size_t)H * W);
    int bad = 0;
    if (!a || !b) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    const int64_t ka = oracle_cclremsp(img, H, W, W, conn, a);
    const int64_t kb = oracle_paremsp_threads(img, H, W, W, conn, b, threads);
    if (ka != kb || memcmp(a, b, sizeof(int32_t) * (size_t)H * W) != 0) {
        printf("FAIL %s %dx%d conn %d threads %d: K %lld vs %lld\n", what, H, W, conn, threads, (long long)ka,
               (long long)kb);
        bad = 1;
    }
    free(a);
    free(b);
    return bad;
}

int main(void)
{
    static const int shapes[][2] = {{37, 53}, {64, 64}, {129, 200}, {256, 317}, {401, 150}};
    static const int dens[] = {30, 45, 50, 59, 70};
    static const int threads[] = {2, 3, 4, 8, 16};
    int cases = 0, failures = 0;
    for (size_t si = 0; si < sizeof(shapes) / sizeof(shapes[0]); si++) {
        const int H = shapes[si][0], W = shapes[si][1];
        uint8_t *img = malloc((size_t)H * W);
        for (size_t di = 0; di < sizeof(dens) / sizeof(dens[0]); di++) {
            for (int i = 0; i < H * W; i++)
                img[i] = (uint8_t)((rnd() % 100) < (uint32_t)dens[di]);
            for (int conn = 4; conn <= 8; conn += 4)
                for (size_t ti = 0; ti < sizeof(threads) / sizeof(threads[0]); ti++) {
                    failures += check(img, H, W, conn, threads[ti], "random");
                    cases++;
                }
        }
        /* bars: every other row full, joined by one column; a comb */
        for (int r = 0; r < H; r++)
            for (int c = 0; c < W; c++)
                img[r * W + c] = (uint8_t)((r % 2 == 0) || c == W / 2);
        for (int conn = 4; conn <= 8; conn += 4)
            for (size_t ti = 0; ti < sizeof(threads) / sizeof(threads[0]); ti++) {
                failures += check(img, H, W, conn, threads[ti], "bars");
                cases++;
            }
        for (int r = 0; r < H; r++)
            for (int c = 0; c < W; c++)
                img[r * W + c] = (uint8_t)((c % 2 == 0 && r < H - 1) || r == H - 1);
        for (int conn = 4; conn <= 8; conn += 4)
            for (size_t ti = 0; ti < sizeof(threads) / sizeof(threads[0]); ti++) {
                failures += check(img, H, W, conn, threads[ti], "comb");
                cases++;
            }
        free(img);
    }
    printf("%d cases, %d failures\n", cases, failures);
    return failures ? 1 : 0;
}

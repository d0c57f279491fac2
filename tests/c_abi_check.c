/* Calls libnbody's host-only entry points from plain C (no GPU needed): the header compiles as
 * C, the library links, and parameter validation answers through the C ABI. */
#include <stdio.h>
#include <string.h>

#include "nbody.h"

int main(void)
{
    nb_params p;
    memset(&p, 0, sizeof p);
    p.n = 2048;
    p.n1 = 1366;
    p.G = 1.0;
    p.m = 1.5 / 2048.0;
    p.dt = 1e-4;
    p.D1 = 0.0489;
    p.D2 = 0.0411;
    p.q = 0.5;
    p.a = 1.0;
    p.R2_0 = 0.2;
    p.growth_rate = 1e-4;
    p.growth_on = 1;
    p.mode = NB_FP32_KAHAN;
    p.law = NB_LAW_CONTACT;
    size_t bytes = 0;
    int rc = nb_scratch_bytes(&p, &bytes);
    printf("scratch %d %zu\n", rc, bytes);
    p.law = NB_LAW_PAPER;
    p.eps = 0.005;
    p.gamma = 10.0;
    p.beta = 0.5;
    size_t bytes_paper = 0;
    rc = nb_scratch_bytes(&p, &bytes_paper);
    printf("paper %d %zu\n", rc, bytes_paper);
    p.mode = NB_FP32_PLAIN;
    rc = nb_scratch_bytes(&p, &bytes);
    printf("plain-paper %d %s\n", rc, nb_strerror(rc));
    int32_t ki = 0, ns = 0, ib = 0, jc = 0, rows = 0;
    rc = nb_tile_config(262144, 201650, NB_FP32_KAHAN, NB_LAW_CONTACT, &ki, &ns, &ib, &jc, &rows);
    printf("tile %d %d %d %d %d %d\n", rc, ki, ns, ib, jc, rows);
    printf("version %d\n", nb_version());
    nb_system *s = NULL;
    rc = nb_create(NULL, NULL, NULL, &s);
    printf("create-null %d %s\n", rc, s == NULL ? "null" : "set");
    return 0;
}

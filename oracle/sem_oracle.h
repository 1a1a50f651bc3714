/*
 * sem_oracle.h -- interface of the plain FP64 CPU reference (test
 * infrastructure only; the product library never includes or links it).
 */
#ifndef SEM_ORACLE_H
#define SEM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_MAP_BOX = 0, ORC_MAP_PIPE = 1 };

typedef struct {
    int N;                  /* polynomial order, N+1 GLL points per direction   */
    int nel[3];             /* elements along x, y, z                           */
    int periodic[3];        /* 1 = periodic along that axis                     */
    double lo[3], hi[3];    /* box extent (pipe: square cross-section and z)    */
    int mapping;            /* ORC_MAP_BOX or ORC_MAP_PIPE                      */
    const double *vertices; /* optional (nx+1)(ny+1)(nz+1)*3 vertex lattice      */
    int dirichlet;          /* bit 2d / 2d+1: low / high face of axis d          */
} orc_mesh;

typedef struct {
    int N;
    long ne, nloc, nglob;
    const double *D, *G, *h1, *h2, *B;
    const int64_t *gid;
    const uint8_t *gmask;
    const double *invdiag;
} orc_problem;

typedef struct {
    int iterations;
    int restarts;
    double rel_residual;
    double bnorm;
} orc_pcg_stats;

void orc_gll(int N, double *xi, double *w);
void orc_deriv(int N, const double *xi, double *D);
long orc_num_elements(const orc_mesh *m);
long orc_num_local(const orc_mesh *m);
long orc_num_global(const orc_mesh *m);
void orc_coords(const orc_mesh *m, const double *xi, const long *elems, long ne,
                double *x, double *y, double *z);
void orc_geom(const orc_mesh *m, const double *w, const double *D, const long *elems, long ne,
              const double *x, const double *y, const double *z, double *G, double *B);
void orc_numbering(const orc_mesh *m, const long *elems, long ne, int64_t *gid);
void orc_global_mask(const orc_mesh *m, uint8_t *gmask);
void orc_multiplicity(long nloc, const int64_t *gid, long nglob, int32_t *gmult);
void orc_ax(int N, long ne, const double *D, const double *G, const double *h1,
            const double *h2, const double *B, const double *u, double *w);
void orc_gs(long nloc, const int64_t *gid, long nglob, const uint8_t *gmask, double *v);
void orc_jacobi(int N, long ne, const double *D, const double *G, const double *h1,
                const double *h2, const double *B, const int64_t *gid, long nglob,
                const uint8_t *gmask, double *invdiag);
void orc_apply(const orc_problem *pb, const double *v, double *w);
int orc_threads(int n);
int orc_pcg(const orc_problem *pb, const double *b, double *x, double tol, int max_iter,
            orc_pcg_stats *st);

#ifdef __cplusplus
}
#endif
#endif

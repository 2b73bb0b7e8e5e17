/*
 * spinlat_oracle.h -- declarations of the CPU oracle (test infrastructure only;
 * see spinlat_oracle.c for what each function follows in the paper).
 * The oracle has its own parameter struct and shares nothing with the GPU
 * library's public header.
 */
#ifndef SPINLAT_ORACLE_H
#define SPINLAT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_ABI 1
#define OR_ISING 0
#define OR_NORTH_EAST 1
#define OR_NE_TILES 2   /* North-East model, paper's random sub-lattice algorithm */
#define OR_NE_BALANCED 3 /* its balanced variant: red, then white sites */
#define OR_NE_COUPLED 4  /* NE constraint on the Ising energy (J, h, T): Sec. 3.2, J != 0 */
#define OR_INIT_COLD 0
#define OR_INIT_RANDOM 1
#define OR_TAG_SWEEP 0u
#define OR_TAG_INIT 1u
#define OR_TAG_NE_TILES 2u
#define OR_TAG_NE_BALANCED 3u
#define OR_RECORD_WORDS 5

typedef struct {
    int32_t model;   /* OR_ISING, OR_NORTH_EAST, OR_NE_TILES, OR_NE_BALANCED, OR_NE_COUPLED */
    int32_t dim;     /* 2 or 3 (NE: 2) */
    int32_t L;       /* even */
    int32_t two_s;   /* 1: s in {-1,+1}; 2: s in {-1,0,+1} */
    int32_t init;    /* OR_INIT_COLD / OR_INIT_RANDOM (Ising) */
    int32_t pad;
    double J, h, T;  /* Ising and OR_NE_COUPLED */
    double c;        /* NE up-density, 0 < c < 1 (OR_NE_COUPLED: initial state only) */
    uint64_t seed;
    int32_t tile;    /* OR_NE_TILES: side B of the square sub-lattices */
    int32_t lambda;  /* OR_NE_TILES: sites updated together per iteration */
} or_params;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint32_t or_rand(uint64_t seed, uint32_t tag, uint32_t t, uint32_t colour,
                 uint64_t k, int w, int j);
uint64_t or_threshold_from_prob(double p);
uint64_t or_threshold(double dE, double T);
double or_delta_e(double J, double h, int s, int sp, int nsum);
int64_t or_nsites(const or_params* p);
void or_init(const or_params* p, int8_t* s);
int64_t or_half_sweep(const or_params* p, int8_t* s, uint32_t t, uint32_t colour);
void or_recount(const or_params* p, const int8_t* s, int64_t out[3]);
void or_reset_persistence(const or_params* p, int8_t* s);
int or_run(const or_params* p, int8_t* s, uint32_t t0, uint32_t nsweeps,
           int64_t* records, int nthreads);
int64_t or_threshold_table(const or_params* p, uint64_t* out, int64_t cap);
int64_t or_ne_tiles_launch(const or_params* p, const int8_t* src, int8_t* dst, uint32_t launch);
int64_t or_ne_balanced_launch(const or_params* p, const int8_t* src, int8_t* dst, uint32_t launch);
int or_abi(void);

#ifdef __cplusplus
}
#endif
#endif

/* Internal state of the CPU oracle.  TEST INFRASTRUCTURE ONLY. */
#ifndef ISC_ORACLE_MODEL_H
#define ISC_ORACLE_MODEL_H
#include <vector>
#include "oracle.h"

struct orc_perf {
    int32_t cell;
    int32_t kind;     /* 1 producer, 2 injector, 3 controlled producer, 4 controlled injector */
    int32_t well;     /* kinds 3/4: index into orc_model::cw, else -1 */
    double wi;        /* Peaceman well index, m^3 */
    double bhp;       /* producer */
    double q[ORC_NSPEC];  /* injector molar rates per species, mol/s */
    double qE;        /* injector energy rate, W */
    double q_total;   /* injector total molar rate (for sensitivity) */
};

/* a well whose bottom-hole pressure is an unknown (kinds 3, 4) */
struct orc_cwell {
    int32_t kind, control;
    double target, limit;
    double z[ORC_NSPEC], Hinj;   /* injector: composition and molar enthalpy at T_inj */
    int32_t p0 = 0, np = 0;      /* its perforations: perfs[p0 .. p0 + np) */
    int32_t c0 = 0;              /* their first index among the controlled wells' perforations */
    double bhp = 0.0;            /* state: bottom-hole pressure, Pa */
    int32_t on_limit = 0;        /* state: rate control suspended at the BHP limit */
};

struct orc_model {
    orc_grid g;
    orc_fluid fl;
    int32_t n;                    /* cells */
    std::vector<double> logk, kh, kz, poro;
    double kvkh;
    std::vector<int32_t> row_ptr, col_idx, diag_pos;
    std::vector<orc_perf> perfs;
    std::vector<orc_well> wells_in;        /* shallow copies for WI recompute */
    std::vector<std::vector<int32_t>> well_cells;
    std::vector<orc_cwell> cw;            /* controlled wells, in input order */
    int32_t heater_cell = -1;     /* a heat source in one cell's energy balance (W), or none */
    double heater_W = 0.0;
};

namespace orc {
/* neighbour list helpers */
int32_t block_of(const orc_model& m, int32_t i, int32_t j);  /* index into J or -1 */
double cell_volume(const orc_model& m);
double depth(const orc_model& m, int32_t i);
void compute_wells(orc_model& m);
}
#endif

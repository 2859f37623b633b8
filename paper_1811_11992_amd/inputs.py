"""Seeded synthetic inputs and the SI physics card.

This module holds data only: the fluid, rock and reaction parameters of the
paper's combustion-tube model (Section 4.1, tables "Input data for tube model"
and the reaction/well table) converted to SI units, synthesised relative-
permeability tables, Cartesian grids, permeability and porosity fields, wells
and initial states.  It contains none of the simulator's arithmetic (no
property correlation, residual, Jacobian or solver step) and is the only
module that both the GPU library and the CPU oracle consume.

Species order (7): 0 W (water), 1 LO (light oil), 2 HO (heavy oil),
3 O2, 4 CO2, 5 N2, 6 coke.  The inert gas "IR" of the paper is split into CO2
(the only carbon-oxide reaction product) and N2 (inert, injected with air).

Primary unknowns per cell (8), in this order:
    p, x_LO, y_O2, y_CO2, T, S_w, S_g, C_c
Equation rows per cell (8), in this order:
    W, LO, HO, O2, CO2, N2 molar balances, energy, coke.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np

# --------------------------------------------------------------------------
# Unit conversions (exact or standard factors)
# --------------------------------------------------------------------------
PSI = 6894.757293168361          # Pa per psi
LBMOL_FT3 = 16018.46337396014    # mol/m3 per lbmol/ft3
BTU_LBMOL = 2.326                # J/mol per Btu/lbmol (IT Btu)
BTU_LBMOL_R = 4.1868             # J/(mol K) per Btu/(lbmol R)
DAY = 86400.0                    # s per day
CP = 1.0e-3                      # Pa s per cP
MD = 9.869233e-16                # m2 per millidarcy
FT = 0.3048                      # m per ft
BTU = 1055.05585262              # J per Btu (IT)
R_GAS = 8.314462618              # J/(mol K)


def degF_to_K(tf: float) -> float:
    return (tf + 459.67) / 1.8


NSPEC = 7      # W LO HO O2 CO2 N2 coke
NGAS = 6       # species that may be in the gas phase
NREAC = 4
NUNK = 8
NTAB = 101     # rows of the SWT / SLT tables, knots at S = k/100

# unknown indices
P, XLO, YO2, YCO2, T, SW, SG, CC = range(8)
UNKNOWN_NAMES = ("p", "x_LO", "y_O2", "y_CO2", "T", "S_w", "S_g", "C_c")
EQUATION_NAMES = ("W", "LO", "HO", "O2", "CO2", "N2", "energy", "coke")


class Fluid(ctypes.Structure):
    """Binary layout of the SI physics card (``isc_fluid`` in include/isc.h).

    Every field is SI.  Correlation coefficients are stored in the form in
    which they are used with T in kelvin and p in pascal.
    """
    _fields_ = [
        ("M", ctypes.c_double * NSPEC),          # kg/mol
        ("Tc", ctypes.c_double * NGAS),          # K
        ("pc", ctypes.c_double * NGAS),          # Pa
        ("rho_ref", ctypes.c_double * 3),        # mol/m3, liquid W, LO, HO
        ("cp_liq", ctypes.c_double * 3),         # 1/Pa   liquid compressibility
        ("ct1_liq", ctypes.c_double * 3),        # 1/K    liquid thermal expansion
        ("rho_coke", ctypes.c_double),           # mol/m3
        ("cpg", ctypes.c_double * (NGAS * 4)),   # cp_c(T) = sum_j cpg[c][j] T^j, J/(mol K)
        ("hvr", ctypes.c_double * 3),            # Hv(T) = hvr (Tc - T)^ev, J/mol, T<Tc
        ("ev", ctypes.c_double * 3),
        ("avisc", ctypes.c_double * 3),          # mu = avisc exp(bvisc / T), Pa s
        ("bvisc", ctypes.c_double * 3),          # K
        ("avg", ctypes.c_double * NGAS),         # mu_g,c = avg T^bvg, Pa s
        ("bvg", ctypes.c_double * NGAS),
        ("kv1", ctypes.c_double * 3),            # K = kv1/p exp(kv4/(T - kv5)); Pa
        ("kv4", ctypes.c_double * 3),            # K
        ("kv5", ctypes.c_double * 3),            # K
        ("stoich", ctypes.c_double * (NREAC * NSPEC)),  # s[R][c], reactants < 0
        ("Afreq", ctypes.c_double * NREAC),      # r1,r2,r4: 1/(Pa s); r3: 1/s
        ("Eact", ctypes.c_double * NREAC),       # J/mol
        ("Hreac", ctypes.c_double * NREAC),      # J/mol of reaction, + exothermic
        ("eps", ctypes.c_double),                # PER correction constant
        ("Ccmax", ctypes.c_double),              # mol/m3 bulk
        ("p_ref", ctypes.c_double),              # Pa
        ("T_ref", ctypes.c_double),              # K
        ("cpor", ctypes.c_double),               # 1/Pa, linear porosity law
        ("cp_rock", ctypes.c_double),            # J/(m3 K) rock volumetric heat capacity
        ("cp_coke", ctypes.c_double),            # J/(mol K)
        ("Kcond", ctypes.c_double * 4),          # W/(m K): water, oil, gas, rock
        ("grav", ctypes.c_double),               # m/s2
        ("Rgas", ctypes.c_double),               # J/(mol K)
        ("krocw", ctypes.c_double),              # k_ro at connate water
        ("krw", ctypes.c_double * NTAB),         # SWT table, indexed by S_w
        ("krow", ctypes.c_double * NTAB),
        ("krg", ctypes.c_double * NTAB),         # SLT table, indexed by S_g
        ("krog", ctypes.c_double * NTAB),
    ]


class Grid(ctypes.Structure):
    """``isc_grid``: cell i = ix + nx*(iy + ny*iz); iz grows with depth."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


WELL_BHP_PRODUCER = 1
WELL_RATE_INJECTOR = 2
WELL_PRODUCER = 3        # bottom-hole pressure as an unknown, with a control
WELL_INJECTOR = 4
# controls of kinds 3/4: BHP, or a molar rate (producer: of the phases in the mask)
CTRL_BHP, CTRL_WATER, CTRL_OIL, CTRL_GAS = 0, 1, 2, 4
CTRL_LIQUID = CTRL_WATER | CTRL_OIL
CTRL_TOTAL = CTRL_WATER | CTRL_OIL | CTRL_GAS
CTRL_RATE = CTRL_TOTAL   # an injector's rate control (any nonzero value)


class Well(ctypes.Structure):
    """``isc_well``: one well with its perforated cells (host pointer)."""
    _fields_ = [("kind", ctypes.c_int32), ("nperf", ctypes.c_int32),
                ("perf_cells", ctypes.POINTER(ctypes.c_int32)),
                ("target", ctypes.c_double),      # BHP in Pa (kind 1, control 0) or mol/s
                ("T_inj", ctypes.c_double),       # K
                ("z_inj", ctypes.c_double * NSPEC),
                ("rw", ctypes.c_double), ("skin", ctypes.c_double),
                ("control", ctypes.c_int32),      # kinds 3/4
                ("limit", ctypes.c_double)]       # kinds 3/4 under rate control: BHP limit, Pa


# --------------------------------------------------------------------------
# Physics card (paper Section 4.1, combustion tube tables, converted to SI)
# --------------------------------------------------------------------------
# Critical data, degF / psi, tube model; CO2 from the field model's IR column
# (which is literally CO2: M 44, Tc 88.03 F, pc 1073 psi); N2 takes the tube IR
# critical data.
_TC_F = {"W": 705.7, "LO": 651.7, "HO": 1138.0, "O2": -181.0, "CO2": 88.03, "N2": -232.0}
_PC_PSI = {"W": 3155.0, "LO": 305.7, "HO": 120.0, "O2": 730.0, "CO2": 1073.0, "N2": 500.0}
_M_G = {"W": 18.0, "LO": 156.7, "HO": 675.0, "O2": 32.0, "CO2": 44.0, "N2": 28.013, "coke": 13.0}
# gas heat-capacity polynomial, Btu/(lbmol R^j), T in absolute Rankine
_CPG = {"W": (7.613, 8.616e-4, 0.0, 0.0),
        "LO": (-1.89, 0.1275, -3.9e-5, 4.6e-9),
        "HO": (-8.14, 0.549, -1.68e-4, 1.98e-8),
        "O2": (6.713, -4.883e-7, 1.287e-6, -4.36e-10),
        "CO2": (7.44, -0.0018, 1.975e-6, -4.78e-10),
        "N2": (7.44, -0.0018, 1.975e-6, -4.78e-10)}
# gas viscosity avg (cP / R^bvg), bvg
_AVG = {"W": (8.822e-6, 1.116), "LO": (2.166e-6, 0.943), "HO": (3.926e-6, 1.102),
        "O2": (2.196e-4, 0.721), "CO2": (2.127e-4, 0.702), "N2": (2.127e-4, 0.702)}
GAS = ("W", "LO", "HO", "O2", "CO2", "N2")
LIQ = ("W", "LO", "HO")


def stoichiometry() -> np.ndarray:
    """Molar stoichiometry s[R][c] (species order W LO HO O2 CO2 N2 coke).

    Tube reactions of the paper with IR -> CO2; the CO2 coefficients of the
    oxidations and the coke coefficient of the cracking reaction are set so that
    the molar masses balance exactly (N M = 0).
    """
    M = np.array([_M_G[k] for k in ("W", "LO", "HO", "O2", "CO2", "N2", "coke")])
    s = np.zeros((NREAC, NSPEC))
    # r1: LO + 14.06 O2 -> a CO2 + 6.58 H2O
    s[0, 1], s[0, 3], s[0, 0] = -1.0, -14.06, 6.58
    s[0, 4] = -(s[0] @ M) / M[4]
    # r2: HO + 60.55 O2 -> b CO2 + 28.34 H2O
    s[1, 2], s[1, 3], s[1, 0] = -1.0, -60.55, 28.34
    s[1, 4] = -(s[1] @ M) / M[4]
    # r3: HO -> 2.154 LO + c coke
    s[2, 2], s[2, 1] = -1.0, 2.154
    s[2, 6] = -(s[2] @ M) / M[6]
    # r4: coke + 1.18 O2 -> d CO2 + 0.55 H2O
    s[3, 6], s[3, 3], s[3, 0] = -1.0, -1.18, 0.55
    s[3, 4] = -(s[3] @ M) / M[4]
    return s


def corey_tables():
    """SWT/SLT tables at S = k/100 (the paper gives none; Corey curves).

    S_wc 0.1, S_orw 0.15, S_org 0.1, S_gc 0, exponents 2, krw_max 0.3,
    krocw 1.0, krg_max 0.6.  k_rg and k_rog are indexed by S_g.
    """
    s = np.arange(NTAB) / (NTAB - 1)
    swc, sorw, sorg, sgc = 0.1, 0.15, 0.1, 0.0
    krocw = 1.0
    krw = 0.3 * np.clip((s - swc) / (1 - swc - sorw), 0, 1) ** 2
    krow = krocw * np.clip((1 - s - sorw) / (1 - swc - sorw), 0, 1) ** 2
    krg = 0.6 * np.clip((s - sgc) / (1 - swc - sorg - sgc), 0, 1) ** 2
    krog = krocw * np.clip((1 - swc - sorg - s) / (1 - swc - sorg), 0, 1) ** 2
    return krocw, krw, krow, krg, krog


def physics_card(**overrides) -> Fluid:
    """Build the SI physics card.  Keyword overrides replace named fields
    (scalars) for special-case tests, e.g. ``Afreq=(0,0,0,0)``."""
    f = Fluid()
    for i, k in enumerate(("W", "LO", "HO", "O2", "CO2", "N2", "coke")):
        f.M[i] = _M_G[k] * 1e-3
    for i, k in enumerate(GAS):
        f.Tc[i] = degF_to_K(_TC_F[k])
        f.pc[i] = _PC_PSI[k] * PSI
        for j in range(4):
            # cp in Btu/(lbmol R) with T_R = 1.8 T_K  ->  J/(mol K) with T_K
            f.cpg[i * 4 + j] = BTU_LBMOL_R * _CPG[k][j] * 1.8 ** j
        a, b = _AVG[k]
        f.avg[i] = a * CP * 1.8 ** b
        f.bvg[i] = b
    rho = {"W": 3.466, "LO": 0.3195, "HO": 0.0914}
    cpl = {"W": 3e-6, "LO": 5e-6, "HO": 5e-6}
    ct1 = {"W": 1.2e-4, "LO": 2.839e-4, "HO": 1.496e-4}
    hvr = {"W": 1657.0, "LO": 1917.0, "HO": 12198.0}
    avisc = {"W": 4.7352e-3, "LO": 4.02e-4, "HO": 4.02e-4}
    bvisc = {"W": 2728.2, "LO": 6121.6, "HO": 6121.6}
    kv1 = {"W": 1.7202e6, "LO": 1.4546e5, "HO": 2.7454e5}
    kv4 = {"W": -6869.59, "LO": -4458.73, "HO": -8424.83}
    kv5 = {"W": -376.64, "LO": -387.78, "HO": -205.69}
    for i, k in enumerate(LIQ):
        f.rho_ref[i] = rho[k] * LBMOL_FT3
        f.cp_liq[i] = cpl[k] / PSI
        f.ct1_liq[i] = ct1[k] * 1.8
        f.ev[i] = 0.38
        # Hv = hvr (dT_F)^ev Btu/lbmol with dT_F = 1.8 dT_K
        f.hvr[i] = BTU_LBMOL * hvr[k] * 1.8 ** 0.38
        f.avisc[i] = avisc[k] * CP
        f.bvisc[i] = bvisc[k] / 1.8
        f.kv1[i] = kv1[k] * PSI
        f.kv4[i] = kv4[k] / 1.8
        f.kv5[i] = (kv5[k] + 459.67) / 1.8
    f.rho_coke = 57.2 * LBMOL_FT3
    s = stoichiometry()
    for r in range(NREAC):
        for c in range(NSPEC):
            f.stoich[r * NSPEC + c] = s[r, c]
    A_field = (7.248e11, 7.248e11, 1.00008e7, 1.00008e4)
    for r in range(NREAC):
        if r == 2:
            f.Afreq[r] = A_field[r] / DAY          # cracking: 1/day -> 1/s
        else:
            f.Afreq[r] = A_field[r] / (PSI * DAY)  # 1/(psi day) -> 1/(Pa s)
    for r, e in enumerate((59450.0, 59450.0, 27000.0, 25200.0)):
        f.Eact[r] = e * BTU_LBMOL
    for r, h in enumerate((2.9075e6, 1.2525e7, 4.0e4, 2.25e5)):
        f.Hreac[r] = h * BTU_LBMOL
    f.eps = 1e-4
    f.Ccmax = 5000.0
    f.p_ref = 101325.0
    f.T_ref = 298.15
    f.cpor = 5e-10
    f.cp_rock = 2.35e6
    f.cp_coke = 4.06 * BTU_LBMOL_R
    for i, kc in enumerate((0.6, 0.13, 0.03, 1.7)):
        f.Kcond[i] = kc
    f.grav = 9.80665
    f.Rgas = 8.314462618
    krocw, krw, krow, krg, krog = corey_tables()
    f.krocw = krocw
    for k in range(NTAB):
        f.krw[k], f.krow[k], f.krg[k], f.krog[k] = krw[k], krow[k], krg[k], krog[k]
    for name, val in overrides.items():
        cur = getattr(f, name)
        if isinstance(cur, ctypes.Array):
            for i, v in enumerate(val):
                cur[i] = v
        else:
            setattr(f, name, val)
    return f


def card_array(f: Fluid) -> np.ndarray:
    """The card as a flat float64 view (its binary layout is all doubles)."""
    return np.frombuffer(bytes(f), dtype=np.float64).copy()


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
P0 = 2014.7 * PSI                 # initial pressure and producer BHP (tube model)
T0 = 300.0                        # K
S0 = (0.178, 0.654, 0.168)        # S_w, S_o, S_g (tube model)
XLO0 = 0.744
YO2_0 = 0.208                     # air with ~1% of the gas taken by vapours
RHO_G0 = 5570.0                   # mol/m3, gas molar density at (P0, T0), used to size injection
T_IGNITE = 700.0
# State of an ignition cell at 700 K: the liquids it would flash are removed
# (water almost gone, light oil largely vaporised) so that the gas-phase mole
# fractions stay below one, and its gas holds no oxygen yet, so that the
# injected air is what burns (a cell full of air at 700 K would burn it within
# a fraction of a second and start Newton far outside its convergence basin).
IGNITION_STATE = dict(xLO=0.2, yO2=0.0, yCO2=0.0, Sw=4e-6, Sg=0.346)
DT_DAYS = 0.1


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    logk: np.ndarray          # [N] ln(k_h / m2)
    kv_over_kh: float
    poro: np.ndarray          # [N]
    wells: list               # list of dicts: kind, cells, target, T_inj, z_inj, control, limit
    u0: np.ndarray            # [8][N] initial state
    dt: float                 # s
    nsteps: int
    seed: int
    # a heat source in one cell's energy balance: dict(cell, rate_W, stop_s) -- on
    # from time 0 until stop_s -- or None
    heater: dict | None = None

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def grid(self) -> Grid:
        return Grid(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz)

    def well_structs(self):
        """ctypes array of Well plus the int32 buffers they point into."""
        keep = []
        arr = (Well * max(1, len(self.wells)))()
        for i, w in enumerate(self.wells):
            cells = np.ascontiguousarray(w["cells"], dtype=np.int32)
            keep.append(cells)
            arr[i].kind = w["kind"]
            arr[i].nperf = len(cells)
            arr[i].perf_cells = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            arr[i].target = w["target"]
            arr[i].T_inj = w.get("T_inj", T0)
            z = w.get("z_inj", (0, 0, 0, 0, 0, 0, 0))
            for c in range(NSPEC):
                arr[i].z_inj[c] = z[c]
            arr[i].rw = w.get("rw", 0.1)
            arr[i].skin = w.get("skin", 0.0)
            arr[i].control = w.get("control", 0)
            arr[i].limit = w.get("limit", 0.0)
        return arr, keep


def cell_index(nx, ny, ix, iy, iz):
    return ix + nx * (iy + ny * iz)


def initial_state(nx, ny, nz, ignition_cells=()) -> np.ndarray:
    n = nx * ny * nz
    u = np.empty((NUNK, n))
    u[P] = P0
    u[XLO] = XLO0
    u[YO2] = YO2_0
    u[YCO2] = 0.0
    u[T] = T0
    u[SW] = S0[0]
    u[SG] = S0[2]
    u[CC] = 0.0
    for c in ignition_cells:
        u[T, c] = T_IGNITE
        u[XLO, c] = IGNITION_STATE["xLO"]
        u[YO2, c] = IGNITION_STATE["yO2"]
        u[YCO2, c] = IGNITION_STATE["yCO2"]
        u[SW, c] = IGNITION_STATE["Sw"]
        u[SG, c] = IGNITION_STATE["Sg"]
    return u


def lognormal_logk(rng, size, sigma, mean_md=500.0):
    """ln k (m2) with arithmetic mean ``mean_md`` mD: ln k ~ N(ln m - s^2/2, s^2)."""
    mu = math.log(mean_md * MD) - 0.5 * sigma * sigma
    return mu + sigma * rng.standard_normal(size)


def _air_rate(n_cells_pv: float) -> float:
    """Air injection of 1% of a pore volume per day at RHO_G0, mol/s."""
    return 0.01 * n_cells_pv * RHO_G0 / DAY


# Pore volume one injector perforation serves: a 20 x 20 pattern element of one
# layer.  Sizing the injection per perforation keeps the volume injected per
# step into a perforated cell (about 0.4 of its pore volume at 0.1 day) the
# same on every grid; sizing it on the whole reservoir would push tens of pore
# volumes per step through the injector cells of the 2M- and 9.6M-cell grids.
PATTERN_CELLS = 400


def _perf_air_rate(mean_cell_pv: float, nperf: int) -> float:
    return _air_rate(PATTERN_CELLS * mean_cell_pv) * nperf


AIR = (0.0, 0.0, 0.0, 0.21, 0.0, 0.79, 0.0)


def _wells_corner_columns(nx, ny, nz, mean_cell_pv):
    inj = [cell_index(nx, ny, 0, 0, iz) for iz in range(nz)]
    prod = [cell_index(nx, ny, nx - 1, ny - 1, iz) for iz in range(nz)]
    return [dict(kind=WELL_RATE_INJECTOR, cells=inj, target=_perf_air_rate(mean_cell_pv, len(inj)),
                 T_inj=T0, z_inj=AIR),
            dict(kind=WELL_BHP_PRODUCER, cells=prod, target=P0)]


def _channels(rng, logk3, nchan, width=4, thick=2, kchan_md=100 * 500.0):
    """Overwrite ``logk3[iz, iy, ix]`` with sinusoidal high-permeability channels
    running along x (amplitude 5-20 cells, wavelength 50-150 cells)."""
    nz, ny, nx = logk3.shape
    ix = np.arange(nx)
    lk = math.log(kchan_md * MD)
    for _ in range(nchan):
        amp = rng.uniform(5, 20)
        wl = rng.uniform(50, 150)
        ph = rng.uniform(0, 2 * math.pi)
        y0 = rng.uniform(0, ny)
        z0 = int(rng.integers(0, max(1, nz - thick + 1)))
        yc = y0 + amp * np.sin(2 * math.pi * ix / wl + ph)
        for dzl in range(thick):
            iz = z0 + dzl
            if iz >= nz:
                continue
            for w in range(width):
                iy = np.floor(yc - width / 2 + w).astype(int)
                ok = (iy >= 0) & (iy < ny)
                logk3[iz, iy[ok], ix[ok]] = lk


def make_workload(name: str, nsteps: int | None = None) -> Workload:
    """The five configurations (C1..C5), the combustion tube ("TUBE"), small test
    grids ("tiny:NXxNYxNZ") and small grids with controlled wells ("CW:NXxNYxNZ")."""
    dx, dy, dz = 5.0, 5.0, 2.0
    dt = DT_DAYS * DAY
    if name == "C1":
        seed, nx, ny, nz = 1811, 20, 20, 1
        rng = np.random.Generator(np.random.PCG64(seed))
        n = nx * ny * nz
        logk = lognormal_logk(rng, n, 0.5)
        kvkh = 1.0
        poro = np.full(n, 0.30)
        pv = float(poro.sum()) * dx * dy * dz
        wells = [dict(kind=WELL_RATE_INJECTOR, cells=[cell_index(nx, ny, 0, 0, 0)],
                      target=_air_rate(pv), T_inj=T0, z_inj=AIR),
                 dict(kind=WELL_BHP_PRODUCER, cells=[cell_index(nx, ny, nx - 1, ny - 1, 0)],
                      target=P0)]
        u0 = initial_state(nx, ny, nz, [0])
        steps = 10
    elif name in ("C2", "C4"):
        seed, nx, ny, nz = 11992, 60, 60, 10
        rng = np.random.Generator(np.random.PCG64(seed))
        n = nx * ny * nz
        layer = lognormal_logk(rng, nz, 1.0)
        logk = np.repeat(layer, nx * ny)
        kvkh = 0.1
        poro = rng.uniform(0.25, 0.35, n)
        cpv = float(poro.mean()) * dx * dy * dz
        wells = _wells_corner_columns(nx, ny, nz, cpv)
        u0 = initial_state(nx, ny, nz, [0])
        steps = 50 if name == "C2" else 20
    elif name in ("C3", "C5"):
        if name == "C3":
            seed, nx, ny, nz, nchan = 2018, 200, 200, 50, 24
        else:
            seed, nx, ny, nz, nchan = 355, 400, 400, 60, 96
        rng = np.random.Generator(np.random.PCG64(seed))
        n = nx * ny * nz
        logk3 = lognormal_logk(rng, n, 2.0).reshape(nz, ny, nx)
        _channels(rng, logk3, nchan)
        logk = logk3.reshape(-1).copy()
        kvkh = 0.1
        poro = rng.uniform(0.25, 0.35, n)
        cpv = float(poro.mean()) * dx * dy * dz
        if name == "C3":
            wells = _wells_corner_columns(nx, ny, nz, cpv)
            ign = [0]
        else:
            injxy = [(100, 100), (100, 300), (300, 100), (300, 300)]
            prodxy = [(a, b) for a in (0, 200, 399) for b in (0, 200, 399)]
            q = _perf_air_rate(cpv, nz)
            wells = [dict(kind=WELL_RATE_INJECTOR,
                          cells=[cell_index(nx, ny, a, b, iz) for iz in range(nz)],
                          target=q, T_inj=T0, z_inj=AIR) for a, b in injxy]
            wells += [dict(kind=WELL_BHP_PRODUCER,
                           cells=[cell_index(nx, ny, a, b, iz) for iz in range(nz)],
                           target=P0) for a, b in prodxy]
            ign = [cell_index(nx, ny, a, b, 0) for a, b in injxy]
        u0 = initial_state(nx, ny, nz, ign)
        steps = 10
    elif name == "TUBE":
        # The combustion tube of Section 4.1 (tables "Input data for tube model"):
        # 0.1602 ft x 0.1602 ft x 2.6458 ft in 12 cells stacked vertically,
        # k = 12,700 mD, phi = 0.4142; initially 2014.7 psi, 100 F, saturations
        # (0.178, 0.654, 0.168), x_LO = 0.744 and air in the gas; air injected
        # into the top cell at 0.554 ft3/hr at standard conditions (60 F,
        # 14.696 psia) and 70 F, fluids produced from the bottom cell at a
        # bottom-hole pressure of 2014.7 psi, both wells with the table's well
        # index, and a heater of 4800 Btu/day in the top cell for the first
        # 0.0208333 day.  One-minute steps; the heater's 30 minutes are the
        # first 30.
        seed, nx, ny, nz = 0, 1, 1, 12
        dx = dy = 0.1602 * FT
        dz = 2.6458 * FT / nz
        n = nz
        logk = np.full(n, math.log(12700.0 * MD))
        kvkh = 1.0
        poro = np.full(n, 0.4142)
        t_std, p_std = degF_to_K(60.0), 14.696 * PSI
        q_air = p_std * (0.554 * FT ** 3) / (R_GAS * t_std) / 3600.0      # mol/s
        # The table's well index, 5.54 ft md, for both wells.  The wells take a
        # Peaceman index 2 pi dz k / (ln(r_e / r_w) + skin); the skin that gives
        # the table's value carries it (the tube's cells are narrower than a
        # wellbore, so the geometric part alone does not apply).
        wi = 5.54 * FT * MD
        r_e = 0.14 * math.sqrt(dx * dx + dy * dy)
        skin = 2 * math.pi * dz * 12700.0 * MD / wi - math.log(r_e / 0.1)
        wells = [dict(kind=WELL_RATE_INJECTOR, cells=[0], target=q_air, T_inj=degF_to_K(70.0), z_inj=AIR,
                      skin=skin),
                 dict(kind=WELL_BHP_PRODUCER, cells=[n - 1], target=2014.7 * PSI, skin=skin)]
        u0 = initial_state(nx, ny, nz, [])
        u0[T] = degF_to_K(100.0)
        dt = 60.0
        steps = 40
        heater = dict(cell=0, rate_W=4800.0 * BTU / DAY, stop_s=0.02083333333 * DAY)
        return Workload(name=name, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, logk=logk, kv_over_kh=kvkh,
                        poro=poro, wells=wells, u0=u0, dt=dt, nsteps=nsteps if nsteps is not None else steps,
                        seed=seed, heater=heater)
    elif name.startswith("CW:"):
        # Wells whose bottom-hole pressure is an unknown (well-modelling
        # subsection) on a small grid: a column injector at (0, 0) holding
        # the air rate of the small grids up to a maximum BHP of P0 + 5 MPa,
        # and a column producer at the far corner holding a total molar rate
        # of 0.3 times that down to a minimum BHP of 0.8 P0.  Tests change
        # the controls, targets and limits in the well dicts.
        dims = name.split(":")[1]
        nx, ny, nz = (int(v) for v in dims.split("x"))
        base = make_workload("tiny:" + dims, nsteps)
        pv = float(base.poro.sum()) * dx * dy * dz
        q = _air_rate(pv)
        base.wells = [dict(kind=WELL_INJECTOR, cells=[cell_index(nx, ny, 0, 0, k) for k in range(nz)],
                           target=q, T_inj=T0, z_inj=AIR, control=CTRL_RATE, limit=P0 + 5.0e6),
                      dict(kind=WELL_PRODUCER, cells=[cell_index(nx, ny, nx - 1, ny - 1, k) for k in range(nz)],
                           target=0.3 * q, control=CTRL_TOTAL, limit=0.8 * P0)]
        base.name = name
        return base
    elif name.startswith("tiny:"):
        dims = name.split(":")[1]
        nx, ny, nz = (int(v) for v in dims.split("x"))
        seed = 7 + nx * 10000 + ny * 100 + nz
        rng = np.random.Generator(np.random.PCG64(seed))
        n = nx * ny * nz
        logk = lognormal_logk(rng, n, 0.5)
        kvkh = 0.1
        poro = rng.uniform(0.25, 0.35, n)
        pv = float(poro.sum()) * dx * dy * dz
        if n >= 2:
            wells = [dict(kind=WELL_RATE_INJECTOR, cells=[0], target=_air_rate(pv),
                          T_inj=T0, z_inj=AIR),
                     dict(kind=WELL_BHP_PRODUCER, cells=[n - 1], target=P0)]
        else:
            wells = []
        u0 = initial_state(nx, ny, nz, [0] if n >= 2 else [])
        steps = 3
    else:
        raise ValueError(f"unknown workload {name!r}")
    return Workload(name=name, nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, logk=logk,
                    kv_over_kh=kvkh, poro=poro, wells=wells, u0=u0, dt=dt,
                    nsteps=nsteps if nsteps is not None else steps, seed=seed)


def random_states(wl: Workload, seed: int, spread: float = 1.0) -> np.ndarray:
    """Random physically admissible states around the initial state, for
    per-kernel parity and Jacobian checks (p, T, saturations and mole fractions
    perturbed; coke positive)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = wl.ncell
    u = np.empty((NUNK, n))
    u[P] = P0 * (1 + spread * rng.uniform(-0.05, 0.1, n))
    u[XLO] = rng.uniform(0.3, 0.9, n)
    u[YO2] = rng.uniform(0.02, 0.2, n)
    u[YCO2] = rng.uniform(0.0, 0.15, n)
    u[T] = T0 + spread * rng.uniform(0.0, 250.0, n)
    u[SW] = rng.uniform(0.12, 0.3, n)
    u[SG] = rng.uniform(0.1, 0.3, n)
    u[CC] = spread * rng.uniform(0.0, 800.0, n)
    return u

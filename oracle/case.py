"""Problem description for the oracle (test infrastructure only)."""
from dataclasses import dataclass

ZBC_PERIODIC, ZBC_NOSLIP, ZBC_WALLMODEL = 0, 1, 2
YBC_PERIODIC, YBC_WALL = 0, 1   # y walls take the z walls' treatment (duct, Sec. 4.4)
SGS_NONE, SGS_SMAG, SGS_SMAG_VD, SGS_DSM, SGS_MLP = 0, 1, 2, 3, 4


@dataclass
class Case:
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    zbc: int = ZBC_PERIODIC
    beta: float = 0.0          # tanh stretching parameter, 0 = uniform
    nu: float = 1e-3
    sgs: int = SGS_NONE
    cs: float = 0.17           # Smagorinsky constant for SMAG / SMAG_VD
    implicit_z: bool = False   # Crank-Nicolson in z (Eqs. twostar_imp1d..p_update_imp1d)
    implicit_3d: bool = False  # Crank-Nicolson in x, y and z (Eqs. twostar_imp3d..p_update_imp3d)
    ubulk: float = 0.0         # > 0: constant flow rate in x (Sec. 4.2)
    h_wm: float = 0.0          # wall-model height, 0 = first cell centre
    kappa: float = 0.41
    bconst: float = 5.2
    advection: bool = True     # False only in tests that isolate the viscous operator
    ybc: int = YBC_PERIODIC    # YBC_WALL: walls at y = 0 and y = ly as well (square duct)

    def __post_init__(self):
        if self.ybc == YBC_WALL and (self.zbc == ZBC_PERIODIC or self.implicit_3d):
            raise ValueError("y walls need walls in z and no CN in y")

    @property
    def zperiodic(self):
        return self.zbc == ZBC_PERIODIC

    @property
    def walls(self):
        return self.zbc != ZBC_PERIODIC

    @property
    def ywalls(self):
        return self.ybc == YBC_WALL

"""Layer marching (vertical neighbours inside a chunk read from the staged
chunk) gives bitwise the fields of the default gather path, and so inherits
its oracle parity."""
import numpy as np
import pytest

from paper_1607_03399_amd import inputs
from paper_1607_03399_amd import wdg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,bits,bc,flux", [(1, 64, "rigid", "upwind"), (2, 32, "dirichlet", "central"),
                                            (3, 32, "rigid", "upwind"), (4, 64, "rigid", "upwind"),
                                            (5, 32, "dirichlet", "upwind")])
def test_layer_march_equals_gathers(N, bits, bc, flux):
    # 5 layers: chunks cut columns at varying layers, so both paths are taken
    m = inputs.layered_config(3, 5, 0.3, seed=N)
    out = []
    for march in (False, True):
        s = wdg.Solver(N, bits, device=0)
        s.set_mesh(m.verts, m.wedges)
        s.set_material(m.c, m.rho)
        s.set_boundary(bc)
        s.set_flux(flux)
        s.set_layer_march(march)
        s.add_ricker_source([0.5, 0.4, 0.6], 6.0, 0.05, 1.0)
        U = np.zeros((s.K, 4, s.NPmax))
        U[:, 0] = inputs.gaussian_pulse(s.node_coords(), width=0.25)
        U[:, 2] = 0.3 * inputs.gaussian_pulse(s.node_coords(), centre=(0.3, 0.6, 0.5), width=0.3)
        s.set_fields(U)
        s.step(15, s.stable_dt(0.5))
        out.append(s.get_fields())
        s.close()
    assert np.array_equal(out[0], out[1])

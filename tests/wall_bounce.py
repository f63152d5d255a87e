"""Single-sphere wall collision in a quiescent liquid (Case 1 of Section 4:
the particle-wall bounce tests against Gondret et al.'s experiments).

A sphere starts at rest above the bottom wall, falls through the liquid,
collides and rebounds.  The effective restitution is e = e_wet / e_dry: the
rebound velocity (largest upward velocity after the collision) over the
impact velocity (downward velocity when the gap first falls below the
lubrication range), divided by the dry restitution of the contact model.
The Stokes number of the collision is St = rho_p d u_impact / (9 mu_f).
Varying the liquid viscosity sweeps St; lubrication and added mass switch on
and off.  The experiments' data are not available, so the cases are compared
internally (trend with St) and between the oracle and the GPU path.

Both steppers advance one step per call so that the velocity maximum is
sampled at every step."""
import math

import numpy as np

import workloads

D = 3.0e-3        # steel sphere diameter (m)
RHO_P = 7800.0    # steel density (kg/m^3)
E_DRY = 0.97      # dry restitution of the contact model
KN = 2.0e4        # wall contact stiffness (N/m)
GAP0 = 3.0        # initial gap in diameters
AFTER = 1500      # steps followed after the first contact
MESH = (4, 4, 6)


def case(mu_f, lubrication=True, added_mass=True):
    m = RHO_P * math.pi / 6 * D ** 3
    tc = workloads.contact_time(KN, E_DRY, m)
    L = 8 * D
    prm = workloads.base_params(Lx=L, Ly=L, Lz=12 * D, nx=MESH[0], ny=MESH[1], nz=MESH[2],
                                kn=KN, restitution=E_DRY, mu_f=mu_f,
                                lubrication=1 if lubrication else 0,
                                c_add=0.5 if added_mass else 0.0, top_wall=0, dt=tc / 50,
                                avg_bandwidth=3 * D)
    ncell = int(np.prod(MESH))
    gradp = np.zeros((ncell, 3))
    gradp[:, 2] = prm["gz"] * prm["rho_f"]  # hydrostatic: buoyancy through -V grad p
    return dict(params=prm, x=np.array([[L / 2, L / 2, D / 2 + GAP0 * D]]), v=np.zeros((1, 3)),
                w=np.zeros((1, 3)), d=np.full(1, D), rho=np.full(1, RHO_P),
                U=np.zeros((ncell, 3)), gradp=gradp, dudt=np.zeros((ncell, 3)))


def follow(step_once, prm, max_steps=40000):
    """Advance until AFTER steps past the first contact; returns z(t), vz(t)."""
    zs, vs = [], []
    contact = None
    for k in range(max_steps):
        z, vz = step_once()
        zs.append(z)
        vs.append(vz)
        if contact is None and z - D / 2 < 0.0:
            contact = k
        if contact is not None and k - contact >= AFTER:
            break
    return np.array(zs), np.array(vs)


def restitution(prm, z, v):
    """(effective restitution, Stokes number, impact velocity)."""
    gap = z - D / 2
    hout = prm["lub_out_frac"] * D
    i_in = int(np.argmax(gap < hout))
    vin = -v[i_in]
    vout = v[i_in:].max()
    St = RHO_P * D * vin / (9 * prm["mu_f"])
    return vout / vin / E_DRY, St, vin


def run_oracle(orc, c):
    st = orc.State(c["params"], c["x"], c["v"], c["w"], c["d"], c["rho"], U=c["U"],
                   gradp=c["gradp"], dudt=c["dudt"])
    st.init_accel()

    def once():
        st.run(1, 0)
        return st.x[0, 2], st.v[0, 2]
    return follow(once, c["params"])

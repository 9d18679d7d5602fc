"""Writes c1_freefall.json: the closed-form free fall of the c1 scene.

With F = I the fixed-corotated stress vanishes, C stays 0 and every node
in a particle's stencil carries the same velocity, so one substep of
Algorithm 1 (grid update of Sec. III-A with b = g, then the symplectic G2P
position update) gives v_{k+1} = v_k + g dt and x_{k+1} = x_k + dt v_{k+1}.
After n substeps from rest: v_n = n dt g and x_n - x_0 = g dt^2 n (n + 1) / 2.
Plain arithmetic only; no oracle or GPU code is involved.
"""
import json
import os

g, dt, n = -9.8, 1e-4, 100
out = {
    "scene": "c1: 8,000 particles, 32^3 grid, dt = 1e-4, gravity -9.8 m/s^2, 100 substeps",
    "citation": "Sec. III-A grid update (eq. mls_mpm_grid) and G2P integration "
                "(eq. mls_mpm_g2p_integration); Algorithm 1",
    "dy": g * dt * dt * n * (n + 1) / 2.0,
    "vy": n * dt * g,
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_freefall.json"), "w") as fh:
    json.dump(out, fh, indent=1)
print(out)

"""Named synthetic workloads of the driven-cavity time step.

Each is fully defined by its parameters: grid nodes per side ``n`` (walls
included), Reynolds number, lid speed 1, dt = cfl * h with cfl = 0.5, Poisson
residual tolerance, precision, and the initial vorticity recipe.
"""

WORKLOADS = {
    "cavity64_re1e3_fp64": dict(n=64, re=1000.0, steps=200, tol=1e-10, precision="fp64",
                                init="rest"),
    "cavity1024_re1e4_fp64": dict(n=1024, re=1.0e4, steps=1000, tol=1e-10, precision="fp64",
                                  init="rest"),
    "cavity1024_re3e4_mixed": dict(n=1024, re=3.0e4, steps=1000, tol=1e-10, precision="mixed",
                                   init="rest"),
    "re_sweep6": dict(members=[(5000.0, 256), (10000.0, 512), (15000.0, 768),
                               (20000.0, 1024), (25000.0, 1024), (30000.0, 1024)],
                      steps=1000, tol=1e-10, init="rest"),
    # many small cavities (a parameter scan at low resolution): 16 x 128^2, Re 500..8000
    "re_scan16_small": dict(members=[(500.0 * (k + 1), 128) for k in range(16)],
                            steps=200, tol=1e-10, init="rest"),
    # coarse grids of Sec. 4: 220^2 for Re 5e3 and 1e4, 300^2 for 1.5e4, and 300^2 at 2e4,
    # where the paper found no solution on that grid; dt as in Table tab:grid
    "grid_dependence": dict(members=[(5000.0, 220), (10000.0, 220), (15000.0, 300),
                                     (20000.0, 300)], dt=1e-3, tol=1e-10, init="rest"),
    # the fine-grid side of the same study: 1024^2 at the two Reynolds numbers the
    # paper finds unsteady on 300^2 (Sec. 4)
    "grid_dependence_1024": dict(members=[(15000.0, 1024), (20000.0, 1024)], dt=1e-3, tol=1e-10,
                                 init="rest"),
    # Table tab:grid of Sec. 4: the production runs at 1024^2 with dt = 0.001, run until
    # the Sec. 4 thresholds on RES_psi and RES_omega hold
    "steady_table_1024": dict(members=[(5000.0, 1024), (10000.0, 1024), (15000.0, 1024),
                                       (20000.0, 1024), (25000.0, 1024), (30000.0, 1024)],
                              dt=1e-3, tol=1e-10, init="rest"),
    "cavity4096_re3e4_mixed_noise": dict(n=4096, re=3.0e4, steps=2000, tol=1e-10,
                                         precision="mixed", init="noise",
                                         noise_amplitude=1e-3, noise_seed=0),
}

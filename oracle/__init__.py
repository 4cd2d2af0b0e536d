"""CPU oracle of the factorized shading bake and the factored re-render loss.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library or its Python
binding.  It shares no code with the GPU path; the two meet only on the
seeded inputs from ``synth``.

* ``oracle.bake``    shading points and the Monte Carlo bake (Eq. 6, 7, 9),
                     brute-force ray casting in double precision (C, built by
                     ``oracle.build``);
* ``oracle.render``  factored re-render, photometric loss and its gradient
                     (Eq. 5, 8, 2/15), the emission-masked loss (Eq. 12/15)
                     with the diffuse prior (Eq. 17), trilinear material
                     grid and its adjoint, in numpy float64;
* ``oracle.cache``   the voxel radiance cache: average pooling of observed
                     pixels onto a grid and the nearest-voxel index (Sec. 4.2);
* ``oracle.hashgrid`` the hash-grid material network of Eq. 14 (hash encoding
                     and MLP), forward and backward, in numpy float64;
* ``oracle.emission`` per-triangle emission re-estimation (Eq. 13 with
                     f = 0: the median of the observed pixels), in numpy.
"""

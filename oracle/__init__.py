"""Plain FP64 CPU oracle for the controllability CG method (CMCG) for
time-harmonic Maxwell's equations (Chaumont-Frelet, Grote, Lanteri, Tang).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only the tests, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code, tables or constants with the HIP library.

Modules
-------
refelem   reference P_q tetrahedron from barycentric monomials, exact rationals
mesh      connectivity, affine geometry, face-node matching by coordinates
dg        upwind DG operator (matrix-free) and its probed sparse matrix
timestep  RK2 / RK4, propagators P_psi, P, P* = S P S, filter accumulation
filters   trapezoid and Hermite period filters
cmcg      initialisation, gradient and CG algorithms of Section 2.2
fs        frequency-domain solve and the discrete-periodic exact solve
fw        limiting-amplitude (full wave) iteration of Section 6
multifreq several harmonics of a base frequency in one CMCG solve
refelem2d reference P_q triangle (2-D transverse-magnetic setting)
mesh2d    triangle connectivity and geometry
dg2d      2-D TM upwind DG operator (e, h1, h2); timestep, cmcg, fs and fw
          run on it unchanged (they dispatch on the problem's dimension)
exact2d   exact cavity and plane-wave solutions, energy-norm error

Parity status: every function is pinned by a test under tests/ against a
closed form, an invariant, a brute-force computation or a library routine,
except the 3-D CFL constants (documented as a reading, not a pin).  The 2-D
operator is pinned by the FS error levels that Section 6 prints, and its CFL
constants by the stability limits of the RK schemes.
"""

"""FP64 CPU oracle of Real-time Neural MPC's linearisation path (TEST INFRASTRUCTURE).

This package is a plain, slow, obviously-correct NumPy implementation of what
the GPU path computes.  It exists only to check the GPU path: only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.
The product library never calls it, and it shares no code with the HIP
kernels (only the seeded input generators in ``workload`` feed both).

Modules and the passages they follow (Salzmann et al., "Real-time Neural MPC",
RA-L 2023):

* ``quadrotor``  nominal rigid-body model f_F, eq. (6), Sec. VI; quaternion
                 conventions (Sec. VI, Notation); rotor geometry (Fig. quad_model).
* ``mlp``        residual network f_D and its Jacobian J_D, eq. (7); the local
                 approximation's parameters f_D-bar and J_D, eq. (4).
* ``rk4``        continuity parameters phi-bar_k, A_k, B_k of the QP (Sec. IV-A,
                 eq. (2) and the definitions that follow it) with the first-order
                 local approximation eq. (4); RK4 discretisation (Sec. III); and
                 the exact ("naive") variant of Sec. IV-A.
* ``riccati``    feedback-phase LQ solve of the QP of Sec. IV-A with the quadratic
                 cost of Sec. VI (MPC cost formulation); brute-force KKT check.
* ``train``      residual training: MSE, backpropagation, Adam (Sec. VII).
* ``simulator``  drag-augmented synthetic plant and residual labels (Sec. VII,
                 system identification).
* ``quant``      round-to-bf16 / round-to-e4m3 emulation.
* ``double_integrator``  the runtime workload of Sec. V: double-integrator
                 nominal model, its first-order RK4 linearisation and one
                 real-time iteration (linearise, Riccati, rollout).

Float64 throughout.  Inputs arrive as float32 arrays and are promoted exactly.
"""

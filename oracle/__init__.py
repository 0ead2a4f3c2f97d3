"""Plain FP64 CPU oracle of the coupled HCA time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, constants,
tables or helpers with the HIP library; the only thing both sides consume is
the seeded synthetic input generator, which holds none of the method's
arithmetic.

The oracle is written from the paper (Lai et al., "A scalable solver for a
stochastic, hybrid cellular automaton model of personalized breast cancer
therapy"), section by section:

* ``constants``  Table 1 and the readings of the silent or garbled passages.
* ``lattice``    Eqs. (oxygen) and (chemo) discretised on the voxel lattice:
                 the 7-point zero-flux Laplacian and the implicit-Euler systems,
                 solved exactly (sparse LU) or by SciPy CG (timing only).
* ``pk``         the plasma concentrations of the intravascular module
                 (Eq. intrachemo3 and the linear regime of the fluorouracil
                 model), evaluated in closed form as the paper does.
* ``ode``        Eqs. (odep53), (odevegf), (cellcycle).
* ``philox``     Philox4x64-10 counter-based generator (Salmon et al., SC'11).
* ``ca``         the stochastic cellular automaton of the cellular module
                 (kill / divide / no space, snapshot semantics, higher-phi
                 priority on conflicts).
* ``model``      Algorithm 1: initialisation and one coupled step.
* ``mlp``        FP64 forward/backward of the ODE surrogate network.

Pins (what each function is checked against) are in ``tests/test_oracle_*.py``.
Functions whose result no external fact pins say "parity unpinned" in their
docstring.
"""

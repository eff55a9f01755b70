"""FP64 CPU oracle for the convolution-product expansion (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

Modules
-------
``expansion``  the expansion ``H_m u = sum_k h_k * (w_k . u)`` (eq. 1.4) and
               its adjoint, three ways: direct circular sums (the plain
               definition, section 3.5's convolution), the explicit DFT
               matrices of section 3.5, and a float64 FFT library call.
``dense``      the dense quadrature of the integral operator (eq. 1.1) built
               from its TVIR (introduction, Example 3.1).
``construct``  the L2 projection of section 4.2 (used only by the
               approximation-rate test).
``grads``      gradients of ``0.5 ||H_m u - f||^2`` with respect to ``u`` and
               to the half-spectra of the ``h_k``.
``wavelets``   periodic orthonormal Daubechies wavelets and Meyer's operator
               representation (section 4.5).
``sections``   the sectioned evaluation of Lemma 3.2 as a function of
               per-section spectra, its adjoint and its spectra gradient.
"""
from . import expansion, dense, construct, grads, wavelets, sections  # noqa: F401

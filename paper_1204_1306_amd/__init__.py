"""MI355X-native Wilson-Dirac / domain-decomposition hot path for stochastic
fermion-determinant ratios (Finkenrath, Knechtli, Leder, "Fermions as Global
Correction: the QCD Case").

The compute path lives in the HIP library ``libpsms.so`` (sources in
``csrc/``, C-ABI in ``include/psms.h``); :mod:`.psms` is its thin Python
binding. :mod:`.synth` draws the seeded synthetic inputs. Importing the
package loads nothing; the library is opened on first use of the binding.
"""
__all__ = ["synth", "psms"]

"""ppmpm: MI355X-native hot path of the stabilized implicit material point method for coupled
large-deformation poromechanics (Zhao & Choo, arXiv 1905.00671).

The compute path is the HIP library ``libppmpm.so`` (sources in ``csrc/``); ``binding`` is its
ctypes binding and ``workloads`` builds seeded synthetic problem statements.  Submodules are
imported lazily so that the input generators can be used without a GPU.
"""
__all__ = ["workloads", "binding"]

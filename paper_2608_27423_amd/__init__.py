"""MI355X-native matrix-free Jacobian of the stabilized ALE Navier-Stokes
operator with rotor/stator mortar coupling.

The compute path lives in the HIP library ``libmortarns.so`` (sources in
``csrc/``); ``binding`` marshals arguments to its C-ABI.  Importing the package
loads nothing; ``binding.lib()`` loads the library and raises if it is absent.
"""
__all__ = ["binding", "inputs"]

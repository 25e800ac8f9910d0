"""MI355X-native hybrid VoF/Phase-Field soluble-surfactant step.

Importing the package loads nothing native; `paper_2605_27534_amd.surf`
loads the HIP library (libsurf.so) and fails loudly when it is missing.
"""
__all__ = ["surf", "synth", "configs"]

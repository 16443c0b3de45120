"""Seeded synthetic RGB-D input sequences (inputs only; no model arithmetic)."""
from .scenes import PRESETS, Scene, SceneConfig, preset

__all__ = ["PRESETS", "Scene", "SceneConfig", "preset"]

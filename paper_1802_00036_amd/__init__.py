"""MI355X-native IP-Basic depth completion (Ku, Harakeh & Waslander, 2018)."""
__version__ = "0.1.0"
